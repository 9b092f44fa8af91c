// scqmc_kernels.hip -- gfx950 kernels of the local-energy engine.
//
// Hot path (one continuous-time step of every walker, eq:locE and the CTMC of
// the paper's "SC-MRCI(s)" section; the overlap of eq:ovlp; Dyall local
// energy for eq:nevpt):
//
//   one wave64 per walker.  The neighbours m of a walker n are grouped by
//   their active part x_m = x_n - Ra + Pa (Ra: up to two removed active
//   spin-orbitals, Pa: up to two added ones).  A group's members differ only
//   in their virtual occupation l_m (the SC class).  The wave walks the
//   (Ra, Pa) candidates 64 at a time, one per lane: the lane validates the
//   candidate, counts the group's rows (virtual sets reachable by at most a
//   double excitation) and does the group's reference-table lookups once:
//     l_m empty     : phi0(x_m)                      (reference hash)
//     one virtual   : y-list of x_m, x-lists of x_m-r (one per electron r)
//     two virtuals  : x-list of x_m
//   where the y-list (x-list) of a determinant with one (two) active electrons
//   removed holds the reference determinants it came from.  A wave prefix
//   scan turns the row counts into a flat row space that all 64 lanes sweep;
//   every row yields H_nm (Slater-Condon with phase) and psi(m) = c_l <m|H|phi0>
//   as a short sum over the group's lists, i.e. over reference determinants
//   that are nonzero.  Per-group rate sums come from a segmented scan in
//   registers, so every reduction has a fixed order.
//
//   The next state is drawn by the first-reaction method (Gillespie) at two
//   levels: exponential clocks keyed by (walker, step, x_m) pick a group with
//   probability Gamma_g / Gamma, then clocks keyed by the class pick a row
//   with probability Gamma_m / Gamma_g.  The draw depends only on the set of
//   neighbours, not on the order they are visited in.
#include "scqmc_device.h"

#define WAVE 64
#define WPB 4   // waves (walkers) per 256-thread block

// ---------------------------------------------------------------------------
// per-wave LDS
// ---------------------------------------------------------------------------
struct GroupInfo {
    unsigned long long xkey;
    double phi;           // phi0(x_m) for groups without virtual electrons
    double gam;           // sum over rows of |psi(m)|
    unsigned off, nrows;
    unsigned fam_end[4];  // cumulative rows per kept-subset of the walker's virtuals
    signed char ra[2], pa[2];
    unsigned char vp[2], nra, npa;
};

struct WaveLDS {
    GroupInfo *G;         // [65]; slot 64 is the selected group
    uint2 *lst;           // [65 * NL]
    unsigned char *occ;   // [64]
    unsigned char *hol;   // [64]
    int NL;
};

__host__ __device__ inline size_t wave_lds_bytes(int NL) {
    size_t b = 65 * sizeof(GroupInfo);
    b += 65 * (size_t)NL * sizeof(uint2);
    b += 128;
    return (b + 15) & ~(size_t)15;
}

__device__ inline WaveLDS carve(unsigned char *base, int NL) {
    WaveLDS L;
    L.G = (GroupInfo *)base;
    L.lst = (uint2 *)(base + 65 * sizeof(GroupInfo));
    L.occ = (unsigned char *)(L.lst + 65 * NL);
    L.hol = L.occ + 64;
    L.NL = NL;
    return L;
}

struct WalkerCtx {
    NDet n;
    int vcode[2];    // virtual codes, ascending
    int vs[2];       // virtual electrons per spin
    int e, h;        // active electrons, active holes
    unsigned long long valid;
};

__device__ __forceinline__ unsigned binom012(int n, int k) {
    if (k == 0) return 1u;
    if (n < k) return 0u;
    if (k == 1) return (unsigned)n;
    return (unsigned)(n * (n - 1) / 2);
}

// pair index k -> (i < j), k = j(j-1)/2 + i
__device__ __forceinline__ void pair_decode(unsigned k, int &i, int &j) {
    int jj = (int)((1.0 + sqrt(1.0 + 8.0 * (double)k)) * 0.5);
    while (jj * (jj - 1) / 2 > (int)k) jj--;
    while ((jj + 1) * jj / 2 <= (int)k) jj++;
    j = jj;
    i = (int)k - jj * (jj - 1) / 2;
}

// subset index -> up to two entries of a sorted list (0: none, 1..n: single, then pairs)
__device__ __forceinline__ void decode_subset(long long idx, int n, const unsigned char *list, int &cnt, int out[2]) {
    out[0] = out[1] = -1;
    if (idx == 0) { cnt = 0; return; }
    if (idx <= n) { cnt = 1; out[0] = list[idx - 1]; return; }
    int i, j;
    pair_decode((unsigned)(idx - 1 - n), i, j);
    cnt = 2;
    out[0] = list[i];
    out[1] = list[j];
}

// k-th virtual orbital of spin sg not occupied by the walker -> virtual code
__device__ __forceinline__ int avail_virtual(const DevProblem &P, const WalkerCtx &W, int sg, int k) {
    int a = k;
    for (int i = 0; i < W.n.nv; i++) {
        int c = W.vcode[i];
        if ((c >= P.V) == sg && c - sg * P.V <= a) a++;
    }
    return sg * P.V + a;
}

__device__ __forceinline__ void sort2(int *v, int n) {
    if (n == 2 && v[0] > v[1]) { int t = v[0]; v[0] = v[1]; v[1] = t; }
}

// Set up candidate group (Ra, Pa) = c; returns the number of rows (0: invalid).
// Lookups go to the group's list slots.
__device__ unsigned group_setup(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, long long c, long long nP,
                                GroupInfo &g, uint2 *lst) {
    long long ri = c / nP, pi = c - ri * nP;
    int nra, npa, ra[2], pa[2];
    decode_subset(ri, W.e, L.occ, nra, ra);
    decode_subset(pi, W.h, L.hol, npa, pa);
    int rs[2] = {0, 0}, ps[2] = {0, 0};
    for (int i = 0; i < nra; i++) rs[ra[i] >> 5]++;
    for (int i = 0; i < npa; i++) ps[pa[i] >> 5]++;
    int vp0 = W.vs[0] + rs[0] - ps[0], vp1 = W.vs[1] + rs[1] - ps[1];
    g.nrows = 0;
    if (vp0 < 0 || vp1 < 0 || vp0 + vp1 > 2) return 0;
    unsigned tot = 0;
    for (int km = 0; km < 4; km++) {
        unsigned rows = 0;
        if (km < (1 << W.n.nv)) {
            int k0 = 0, k1 = 0, nk = 0;
            for (int i = 0; i < W.n.nv; i++)
                if ((km >> i) & 1) { nk++; if (W.vcode[i] >= P.V) k1++; else k0++; }
            int a0 = vp0 - k0, a1 = vp1 - k1;
            int rem = nra + (W.n.nv - nk), add = npa + a0 + a1;
            if (a0 >= 0 && a1 >= 0 && rem >= 1 && rem <= 2 && add == rem)
                rows = binom012(P.V - W.vs[0], a0) * binom012(P.V - W.vs[1], a1);
        }
        tot += rows;
        g.fam_end[km] = tot;
    }
    g.nrows = tot;
    if (!tot) return 0;
    unsigned long long x = W.n.key;
    for (int i = 0; i < nra; i++) x &= ~(1ull << ra[i]);
    for (int i = 0; i < npa; i++) x |= 1ull << pa[i];
    g.xkey = x;
    g.ra[0] = (signed char)ra[0]; g.ra[1] = (signed char)ra[1];
    g.pa[0] = (signed char)pa[0]; g.pa[1] = (signed char)pa[1];
    g.nra = (unsigned char)nra; g.npa = (unsigned char)npa;
    g.vp[0] = (unsigned char)vp0; g.vp[1] = (unsigned char)vp1;
    g.gam = 0.0;
    g.phi = 0.0;
    int vp = vp0 + vp1;
    if (vp == 0) {
        uint2 oc = table_find(P.ref, x);
        g.phi = oc.y ? P.ref.vals[oc.x] : 0.0;
    } else if (vp == 2) {
        lst[0] = table_find(P.xtab, x);
    } else {
        lst[0] = table_find(P.ytab, x);
        int k = 1;
        unsigned long long y = x;
        while (y) {
            int r = __ffsll((long long)y) - 1;
            y &= y - 1ull;
            lst[k++] = table_find(P.xtab, x & ~(1ull << r));
        }
    }
    return tot;
}

// <m|H|phi0> for m = y + (virtual s): singles from the y-list, doubles from
// the x-lists of y - r (skipping reference determinants that are singles).
template <class ListFn>
__device__ double phi1(const DevProblem &P, unsigned long long y, int s, ListFn lists) {
    int gs = g_of_virtual(P, s);
    double acc = 0.0;
    NDet d;
    d.nv = 0;
    uint2 oc = lists(0);
    for (unsigned k = 0; k < oc.y; k++) {
        int t = (int)P.ytab.codes[oc.x + k];
        double ph0 = P.ytab.vals[oc.x + k];
        int gt = g_of_active(P, t);
        d.key = y | (1ull << t);
        double v = single_elem(P, d, gt, gs, false);
        acc += phase_single(P, d, gt, gs) * v * ph0;
    }
    unsigned long long yy = y;
    int li = 1;
    while (yy) {
        int r = __ffsll((long long)yy) - 1;
        yy &= yy - 1ull;
        uint2 ox = lists(li++);
        int gr = g_of_active(P, r);
        int Q1 = gs < gr ? gs : gr, Q2 = gs < gr ? gr : gs;
        for (unsigned k = 0; k < ox.y; k++) {
            unsigned code = P.xtab.codes[ox.x + k];
            int t = (int)(code >> 6), u = (int)(code & 63u);
            if (t == r || u == r) continue;
            double ph0 = P.xtab.vals[ox.x + k];
            d.key = (y & ~(1ull << r)) | (1ull << t) | (1ull << u);
            int P1 = g_of_active(P, t), P2 = g_of_active(P, u);
            acc += phase_double(P, d, P1, P2, Q1, Q2) * double_elem(P, P1, P2, Q1, Q2) * ph0;
        }
    }
    return acc;
}

// <m|H|phi0> for m = x + (virtuals s1 < s2), from the x-list of x
__device__ double phi2(const DevProblem &P, unsigned long long x, int s1, int s2, uint2 ox) {
    int Q1 = g_of_virtual(P, s1), Q2 = g_of_virtual(P, s2);
    double acc = 0.0;
    NDet d;
    d.nv = 0;
    for (unsigned k = 0; k < ox.y; k++) {
        unsigned code = P.xtab.codes[ox.x + k];
        int t = (int)(code >> 6), u = (int)(code & 63u);
        double ph0 = P.xtab.vals[ox.x + k];
        d.key = x | (1ull << t) | (1ull << u);
        int P1 = g_of_active(P, t), P2 = g_of_active(P, u);
        acc += phase_double(P, d, P1, P2, Q1, Q2) * double_elem(P, P1, P2, Q1, Q2) * ph0;
    }
    return acc;
}

// psi of one determinant, lookups done here (one lane)
__device__ double psi_direct(const DevProblem &P, unsigned long long key, int nv, const int *vcode) {
    long long cls;
    double phi;
    if (nv == 0) {
        uint2 oc = table_find(P.ref, key);
        return oc.y ? P.ccls[0] * P.ref.vals[oc.x] : 0.0;
    }
    if (nv == 1) {
        cls = class_id1(P.V, vcode[0]);
        phi = phi1(P, key, vcode[0], [&](int k) -> uint2 {
            if (k == 0) return table_find(P.ytab, key);
            unsigned long long y = key;
            for (int i = 1; i < k; i++) y &= y - 1ull;
            int r = __ffsll((long long)y) - 1;
            return table_find(P.xtab, key & ~(1ull << r));
        });
    } else {
        cls = class_id2(P.V, vcode[0], vcode[1]);
        phi = phi2(P, key, vcode[0], vcode[1], table_find(P.xtab, key));
    }
    return P.ccls[cls] * phi;
}

struct RowOut {
    double hnm, psi, hd, phase;
    long long cls;
    unsigned long long key;
    unsigned virt;
    bool ok, same_cls;
};

// Row r of group g: neighbour m, <m|H|n>, psi(m), the Dyall element if m has
// the walker's virtual occupation.
__device__ void eval_row(const DevProblem &P, const WalkerCtx &W, const GroupInfo &g, const uint2 *lst, unsigned r,
                         RowOut &o) {
    int km = 0;
    unsigned start = 0;
    while (r >= g.fam_end[km]) { start = g.fam_end[km]; km++; }
    r -= start;
    int kc[2], nk = 0, k0 = 0, k1 = 0, rmv[2], nrmv = 0;
    for (int i = 0; i < W.n.nv; i++) {
        if ((km >> i) & 1) {
            kc[nk++] = W.vcode[i];
            if (W.vcode[i] >= P.V) k1++; else k0++;
        } else {
            rmv[nrmv++] = W.vcode[i];
        }
    }
    int a0 = (int)g.vp[0] - k0, a1 = (int)g.vp[1] - k1;
    unsigned c1 = binom012(P.V - W.vs[1], a1);
    unsigned i0 = r / c1, i1 = r - i0 * c1;
    int ad[2], nad = 0;
    if (a0 == 1) ad[nad++] = avail_virtual(P, W, 0, (int)i0);
    else if (a0 == 2) { int i, j; pair_decode(i0, i, j); ad[nad++] = avail_virtual(P, W, 0, i); ad[nad++] = avail_virtual(P, W, 0, j); }
    if (a1 == 1) ad[nad++] = avail_virtual(P, W, 1, (int)i1);
    else if (a1 == 2) { int i, j; pair_decode(i1, i, j); ad[nad++] = avail_virtual(P, W, 1, i); ad[nad++] = avail_virtual(P, W, 1, j); }
    int Lp[2], nl = 0;
    for (int i = 0; i < nk; i++) Lp[nl++] = kc[i];
    for (int i = 0; i < nad; i++) Lp[nl++] = ad[i];
    sort2(Lp, nl);
    o.cls = nl == 0 ? 0 : (nl == 1 ? class_id1(P.V, Lp[0]) : class_id2(P.V, Lp[0], Lp[1]));
    o.key = g.xkey;
    o.virt = (nl > 0 ? (unsigned)Lp[0] : SCQ_NOVIRT) | ((nl > 1 ? (unsigned)Lp[1] : SCQ_NOVIRT) << 16);
    o.same_cls = (nad == 0 && nk == W.n.nv);
    // outer excitation n -> m
    int Pr[2], nP = 0, Qa[2], nQ = 0;
    for (int i = 0; i < g.nra; i++) Pr[nP++] = g_of_active(P, g.ra[i]);
    for (int i = 0; i < nrmv; i++) Pr[nP++] = g_of_virtual(P, rmv[i]);
    for (int i = 0; i < g.npa; i++) Qa[nQ++] = g_of_active(P, g.pa[i]);
    for (int i = 0; i < nad; i++) Qa[nQ++] = g_of_virtual(P, ad[i]);
    sort2(Pr, nP);
    sort2(Qa, nQ);
    o.hd = 0.0;
    if (nP == 1) {
        double ph = phase_single(P, W.n, Pr[0], Qa[0]);
        o.phase = ph;
        o.hnm = ph * single_elem(P, W.n, Pr[0], Qa[0], true);
        if (o.same_cls && P.mode == 1) o.hd = ph * single_elem(P, W.n, Pr[0], Qa[0], false);
    } else {
        double ph = phase_double(P, W.n, Pr[0], Pr[1], Qa[0], Qa[1]);
        o.phase = ph;
        o.hnm = ph * double_elem(P, Pr[0], Pr[1], Qa[0], Qa[1]);
        o.hd = o.hnm;
        if (P.eps_screen > 0.0 && !(fabs(o.hnm) > P.eps_screen)) { o.ok = false; o.psi = 0.0; return; }
    }
    double phi;
    if (nl == 0) phi = g.phi;
    else if (nl == 1) phi = phi1(P, g.xkey, Lp[0], [&](int k) -> uint2 { return lst[k]; });
    else phi = phi2(P, g.xkey, Lp[0], Lp[1], lst[0]);
    o.psi = P.ccls[o.cls] * phi;
    o.ok = true;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

__device__ inline void walker_setup(const DevProblem &P, const WaveLDS &L, int lane, unsigned long long key,
                                    unsigned virt, WalkerCtx &W) {
    W.n.key = key;
    W.n.nv = 0;
    W.vs[0] = W.vs[1] = 0;
    unsigned v0 = virt & 0xFFFFu, v1 = virt >> 16;
    if (v0 != SCQ_NOVIRT) { W.vcode[W.n.nv] = (int)v0; W.n.vg[W.n.nv] = g_of_virtual(P, (int)v0); W.vs[v0 >= (unsigned)P.V]++; W.n.nv++; }
    if (v1 != SCQ_NOVIRT) { W.vcode[W.n.nv] = (int)v1; W.n.vg[W.n.nv] = g_of_virtual(P, (int)v1); W.vs[v1 >= (unsigned)P.V]++; W.n.nv++; }
    unsigned long long am = (P.A >= 32) ? 0xFFFFFFFFull : ((1ull << P.A) - 1ull);
    W.valid = am | (am << 32);
    unsigned long long occ = key & W.valid, hol = ~key & W.valid;
    W.e = popc64(occ);
    W.h = popc64(hol);
    unsigned long long below = lane ? ((1ull << lane) - 1ull) : 0ull;
    if ((occ >> lane) & 1ull) L.occ[popc64(occ & below)] = (unsigned char)lane;
    if ((hol >> lane) & 1ull) L.hol[popc64(hol & below)] = (unsigned char)lane;
    __syncwarp();
}

// <n|H|n> (with_virt) or <n|H_0|n> (active only) summed over lanes in a fixed tree
__device__ inline double wave_diag(const DevProblem &P, const WalkerCtx &W, const WaveLDS &L, int lane, bool with_virt) {
    int n = W.e + (with_virt ? W.n.nv : 0);
    double v = 0.0;
    if (lane < n) {
        int gi = lane < W.e ? g_of_active(P, L.occ[lane]) : W.n.vg[lane - W.e];
        int ii = g_idx(P, gi), si = g_spin(P, gi);
        double two = 0.0;
        for (int j = 0; j < n; j++) {
            int gj = j < W.e ? g_of_active(P, L.occ[j]) : W.n.vg[j - W.e];
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

// One walker, one step: local energies, rates and (MOVE) the next state.
template <bool MOVE>
__device__ void walker_eval(const DevProblem &P, const WaveLDS &L, int lane, unsigned long long key, unsigned virt,
                            double psin, uint32_t wid, uint32_t step, EvalOut &out) {
    WalkerCtx W;
    walker_setup(P, L, lane, key, virt, W);
    double hnn = wave_diag(P, W, L, lane, true);
    double hdnn = 0.0;
    bool dy = (P.mode == 1 && W.n.nv > 0);
    if (dy) {
        hdnn = wave_diag(P, W, L, lane, false);
        for (int i = 0; i < W.n.nv; i++) {
            int s = W.vcode[i];
            hdnn += P.eps[s >= P.V ? s - P.V : s];
        }
    }
    long long nR = 1 + W.e + (long long)W.e * (W.e - 1) / 2;
    long long nP = 1 + W.h + (long long)W.h * (W.h - 1) / 2;
    long long ncand = nR * nP;
    double accE = 0.0, accD = 0.0, accG = 0.0;
    double best = INFINITY;
    unsigned long long bestkey = ~0ull;
    long long bestc = -1;
    GroupInfo &mg = L.G[lane];
    uint2 *mlst = L.lst + lane * L.NL;
    for (long long base = 0; base < ncand; base += WAVE) {
        long long c = base + lane;
        unsigned rows = 0;
        if (c < ncand) rows = group_setup(P, W, L, c, nP, mg, mlst);
        else mg.nrows = 0;
        // exclusive scan of row counts
        unsigned inc = rows;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            unsigned o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        mg.off = inc - rows;
        unsigned T = __shfl(inc, WAVE - 1);
        __syncwarp();
        for (unsigned fb = 0; fb < T; fb += WAVE) {
            unsigned f = fb + lane;
            int gi = WAVE;
            double v = 0.0;
            if (f < T) {
                int lo = 0, hi = WAVE - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (L.G[mid].off <= f) lo = mid; else hi = mid - 1;
                }
                gi = lo;
                RowOut o;
                eval_row(P, W, L.G[gi], L.lst + gi * L.NL, f - L.G[gi].off, o);
                if (o.ok) {
                    accE += o.hnm * o.psi;
                    v = fabs(o.psi);
                    accG += v;
                    if (dy && o.same_cls) accD += o.hd * o.psi;
                }
            }
            // segmented inclusive scan of |psi| by group
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                double ov = __shfl_up(v, d);
                int og = __shfl_up(gi, d);
                if (lane >= d && og == gi) v += ov;
            }
            int ng = __shfl_down(gi, 1);
            bool last = (lane == WAVE - 1) || (ng != gi);
            if (last && gi < WAVE) L.G[gi].gam += v;
            __syncwarp();
        }
        if (rows > 0 && mg.gam > 0.0) {
            double tau = exp_draw(P.seed, wid, step, 0u, (uint32_t)mg.xkey, (uint32_t)(mg.xkey >> 32)) / mg.gam;
            if (tau < best || (tau == best && mg.xkey < bestkey)) { best = tau; bestkey = mg.xkey; bestc = c; }
        }
        __syncwarp();
    }
    accE = wave_sum(accE);
    accG = wave_sum(accG);
    if (dy) accD = wave_sum(accD);
    out.eloc = hnn + accE / psin;
    out.elocd = dy ? hdnn + accD / psin : NAN;
    out.gamma = accG / fabs(psin);
    out.moved = false;
    if (!MOVE) return;
    // group of the first reaction
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        double ob = __shfl_xor(best, d);
        unsigned long long ok = __shfl_xor(bestkey, d);
        long long oc = __shfl_xor(bestc, d);
        if (ob < best || (ob == best && ok < bestkey)) { best = ob; bestkey = ok; bestc = oc; }
    }
    if (bestc < 0) return;
    GroupInfo &sg = L.G[WAVE];
    uint2 *slst = L.lst + WAVE * L.NL;
    if (lane == 0) group_setup(P, W, L, bestc, nP, sg, slst);
    __syncwarp();
    unsigned R = sg.nrows;
    double b2 = INFINITY;
    long long bcls = 0x7fffffffffffffffLL;
    double bpsi = 0.0;
    unsigned long long bkey = 0;
    unsigned bvirt = 0;
    for (unsigned r = lane; r < R; r += WAVE) {
        RowOut o;
        eval_row(P, W, sg, slst, r, o);
        if (!o.ok || o.psi == 0.0) continue;
        double tau = exp_draw(P.seed, wid, step, 1u, (uint32_t)o.cls, 0u) / fabs(o.psi);
        if (tau < b2 || (tau == b2 && o.cls < bcls)) { b2 = tau; bcls = o.cls; bpsi = o.psi; bkey = o.key; bvirt = o.virt; }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        double ob = __shfl_xor(b2, d);
        long long oc = __shfl_xor(bcls, d);
        double op = __shfl_xor(bpsi, d);
        unsigned long long ok = __shfl_xor(bkey, d);
        unsigned ov = __shfl_xor(bvirt, d);
        if (ob < b2 || (ob == b2 && oc < bcls)) { b2 = ob; bcls = oc; bpsi = op; bkey = ok; bvirt = ov; }
    }
    __syncwarp();
    if (b2 == INFINITY) return;
    out.moved = true;
    out.psi_new = bpsi;
    out.key_new = bkey;
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
    unsigned long long *key;
    unsigned *virt;
    double *psi;
    double *wsum;                 // [3][W]
    unsigned long long *cacc;     // [4][ncls][2]
    unsigned long long *bad;      // [1]
};

__device__ __forceinline__ long long class_of_virt(const DevProblem &P, unsigned virt) {
    unsigned v0 = virt & 0xFFFFu, v1 = virt >> 16;
    if (v0 == SCQ_NOVIRT) return 0;
    if (v1 == SCQ_NOVIRT) return class_id1(P.V, (int)v0);
    return class_id2(P.V, (int)v0, (int)v1);
}

__global__ __launch_bounds__(256) void k_sample(DevProblem P, WalkerArrays S, long long W, long long step0, int nsteps,
                                                long long burn_in, int NL) {
    extern __shared__ unsigned char smem[];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    long long w = (long long)blockIdx.x * WPB + wave;
    if (w >= W) return;
    WaveLDS L = carve(smem + wave * wave_lds_bytes(NL), NL);
    unsigned long long key = S.key[w];
    unsigned virt = S.virt[w];
    double psi = S.psi[w];
    double st = S.wsum[w], ste = S.wsum[W + w], st0 = S.wsum[2 * W + w];
    long long nbad = 0;
    for (int k = 0; k < nsteps; k++) {
        long long step = step0 + k;
        EvalOut o;
        walker_eval<true>(P, L, lane, key, virt, psi, (uint32_t)w, (uint32_t)step, o);
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
                fx_add(S.cacc + ((long long)lane * P.ncls + cls) * 2, q);
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

// local energies without moving (parity / snapshots)
__global__ __launch_bounds__(256) void k_eval(DevProblem P, const unsigned long long *keys, const unsigned *virts,
                                              const int *valid, long long n, int NL, double *eloc, double *psi_out,
                                              double *gamma, double *elocd, int *cls_out) {
    extern __shared__ unsigned char smem[];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    long long i = (long long)blockIdx.x * WPB + wave;
    if (i >= n) return;
    WaveLDS L = carve(smem + wave * wave_lds_bytes(NL), NL);
    unsigned long long key = keys[i];
    unsigned virt = virts[i];
    int vc[2];
    int nv = 0;
    if ((virt & 0xFFFFu) != SCQ_NOVIRT) vc[nv++] = (int)(virt & 0xFFFFu);
    if ((virt >> 16) != SCQ_NOVIRT) vc[nv++] = (int)(virt >> 16);
    double ps = (valid[i] ? psi_direct(P, key, nv, vc) : 0.0);
    EvalOut o;
    if (ps != 0.0) {
        walker_eval<false>(P, L, lane, key, virt, ps, (uint32_t)i, 0u, o);
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
}

// psi of walkers (initialisation)
__global__ void k_psi(DevProblem P, const unsigned long long *keys, const unsigned *virts, long long n, double *psi) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned virt = virts[i];
    int vc[2];
    int nv = 0;
    if ((virt & 0xFFFFu) != SCQ_NOVIRT) vc[nv++] = (int)(virt & 0xFFFFu);
    if ((virt >> 16) != SCQ_NOVIRT) vc[nv++] = (int)(virt >> 16);
    psi[i] = psi_direct(P, keys[i], nv, vc);
}

// neighbour list of one walker (debug): one wave
__global__ __launch_bounds__(64) void k_neighbors(DevProblem P, unsigned long long key, unsigned virt, int NL,
                                                  long long cap, unsigned long long *okey, unsigned *ovirt,
                                                  signed char *ophase, double *ohnm, double *opsi,
                                                  unsigned long long *count) {
    extern __shared__ unsigned char smem[];
    int lane = threadIdx.x & 63;
    WaveLDS L = carve(smem, NL);
    WalkerCtx W;
    walker_setup(P, L, lane, key, virt, W);
    long long nR = 1 + W.e + (long long)W.e * (W.e - 1) / 2;
    long long nP = 1 + W.h + (long long)W.h * (W.h - 1) / 2;
    long long ncand = nR * nP;
    GroupInfo &mg = L.G[lane];
    uint2 *mlst = L.lst + lane * L.NL;
    for (long long base = 0; base < ncand; base += WAVE) {
        long long c = base + lane;
        unsigned rows = 0;
        if (c < ncand) rows = group_setup(P, W, L, c, nP, mg, mlst);
        for (unsigned r = 0; r < rows; r++) {
            RowOut o;
            eval_row(P, W, mg, mlst, r, o);
            if (!o.ok) continue;
            unsigned long long pos = atomicAdd(count, 1ull);
            if ((long long)pos < cap) {
                okey[pos] = o.key;
                ovirt[pos] = o.virt;
                ophase[pos] = (signed char)(o.phase > 0 ? 1 : -1);
                ohnm[pos] = o.hnm;
                opsi[pos] = o.psi;
            }
        }
        __syncwarp();
    }
}

// ---------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------
// full (pq|rs) = sum_L B_pq B_rs over all N orbitals
__global__ void k_eri_chol(const double *B, int L, long long N2, double *eri) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N2 * N2) return;
    long long pq = i / N2, rs = i - pq * N2;
    double s = 0.0;
    for (int l = 0; l < L; l++) s = fma(B[l * N2 + pq], B[l * N2 + rs], s);
    eri[i] = s;
}

// non-core block, core-folded one-body operator and core energy from the full tensor
__global__ void k_noncore(const double *eri, const double *h1, int N, int C, double *eri_nc, double *heff) {
    int Np = N - C;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long tot = (long long)Np * Np * Np * Np;
    if (i < tot) {
        long long s = i % Np, r = (i / Np) % Np, q = (i / ((long long)Np * Np)) % Np, p = i / ((long long)Np * Np * Np);
        long long NN = N;
        eri_nc[i] = eri[(((C + p) * NN + (C + q)) * NN + (C + r)) * NN + (C + s)];
    }
    if (i < (long long)Np * Np) {
        int p = (int)(i / Np), q = (int)(i % Np);
        long long NN = N;
        double v = h1[(C + p) * NN + (C + q)];
        for (int c = 0; c < C; c++) {
            v += 2.0 * eri[(((C + p) * NN + (C + q)) * NN + c) * NN + c];
            v -= eri[(((C + p) * NN + c) * NN + c) * NN + (C + q)];
        }
        heff[i] = v;
    }
}

__global__ void k_ecore(const double *eri, const double *h1, int N, int C, double e_const, double *out) {
    if (blockIdx.x || threadIdx.x) return;
    long long NN = N;
    double e = e_const;
    for (int i = 0; i < C; i++) e += 2.0 * h1[i * NN + i];
    for (int i = 0; i < C; i++)
        for (int j = 0; j < C; j++)
            e += 2.0 * eri[((i * NN + i) * NN + j) * NN + j] - eri[((i * NN + j) * NN + j) * NN + i];
    *out = e;
}

// table build: expand reference determinants into (key, payload) pairs
// mode 0: the determinant; 1: one active electron removed; 2: two removed
__global__ void k_expand(const unsigned long long *rkeys, long long n, int mode, int per, unsigned long long *okeys,
                         unsigned long long *opay) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long k = rkeys[i];
    if (mode == 0) { okeys[i] = k; opay[i] = (unsigned long long)i << 12; return; }
    int codes[64];
    int ne = 0;
    unsigned long long x = k;
    while (x) { int c = __ffsll((long long)x) - 1; x &= x - 1ull; codes[ne++] = c; }
    long long o = i * per;
    if (mode == 1) {
        for (int a = 0; a < ne; a++) {
            okeys[o + a] = k & ~(1ull << codes[a]);
            opay[o + a] = ((unsigned long long)i << 12) | (unsigned long long)codes[a];
        }
    } else {
        int m = 0;
        for (int a = 0; a < ne; a++)
            for (int b = a + 1; b < ne; b++) {
                okeys[o + m] = k & ~(1ull << codes[a]) & ~(1ull << codes[b]);
                opay[o + m] = ((unsigned long long)i << 12) | ((unsigned long long)codes[a] << 6) | (unsigned long long)codes[b];
                m++;
            }
    }
}

__global__ void k_fill_u64(unsigned long long *p, long long n, unsigned long long v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u32(unsigned *p, long long n, unsigned v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_insert(const unsigned long long *ekeys, long long m, unsigned long long *keys, unsigned long long mask,
                         unsigned *cnt, unsigned *slot_of) {
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    unsigned long long key = ekeys[j];
    unsigned long long slot = scq_hash(key) & mask;
    while (true) {
        unsigned long long prev = atomicCAS(&keys[slot], SCQ_EMPTY_KEY, key);
        if (prev == SCQ_EMPTY_KEY || prev == key) break;
        slot = (slot + 1) & mask;
    }
    atomicAdd(&cnt[slot], 1u);
    slot_of[j] = (unsigned)slot;
}

__global__ void k_assign(const unsigned *cnt, long long cap, unsigned *off, unsigned *total) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    unsigned c = cnt[s];
    off[s] = c ? atomicAdd(total, c) : 0u;
}

__global__ void k_scatter(const unsigned *slot_of, const unsigned long long *epay, long long m, const unsigned *off,
                          unsigned *cur, unsigned long long *tmp) {
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    unsigned s = slot_of[j];
    unsigned pos = off[s] + atomicAdd(&cur[s], 1u);
    tmp[pos] = epay[j];
}

// sort each list by payload (deterministic content order) and write codes / coefficients
__global__ void k_finish(const unsigned *cnt, const unsigned *off, long long cap, unsigned long long *tmp,
                         const double *coeff, uint2 *offcnt, unsigned *codes, double *vals) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    unsigned c = cnt[s], o = off[s];
    offcnt[s] = make_uint2(o, c);
    for (unsigned i = 1; i < c; i++) {
        unsigned long long v = tmp[o + i];
        int j = (int)i - 1;
        while (j >= 0 && tmp[o + j] > v) { tmp[o + j + 1] = tmp[o + j]; j--; }
        tmp[o + j + 1] = v;
    }
    for (unsigned i = 0; i < c; i++) {
        unsigned long long v = tmp[o + i];
        codes[o + i] = (unsigned)(v & 0xFFFull);
        vals[o + i] = coeff[v >> 12];
    }
}

// full determinants [n][2][words] -> (active key, packed virtual codes, valid)
__global__ void k_compact(const unsigned long long *dets, long long n, int words, int N, int C, int A, int na, int nb,
                          unsigned long long *keys, unsigned *virts, int *valid) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long *d = dets + i * 2 * words;
    bool ok = true;
    unsigned long long key = 0;
    int vc[3], nv = 0;
    int V = N - C - A;
    for (int s = 0; s < 2; s++) {
        int cnt = 0;
        for (int p = 0; p < N; p++) {
            int b = (int)((d[s * words + (p >> 6)] >> (p & 63)) & 1ull);
            cnt += b;
            if (p < C) { if (!b) ok = false; }
            else if (p < C + A) { if (b) key |= 1ull << (32 * s + p - C); }
            else if (b) { if (nv < 3) vc[nv] = s * V + (p - C - A); nv++; }
        }
        for (int w = 0; w < words; w++) {   // bits beyond N must be clear
            int lo = 64 * w;
            for (int bbit = 0; bbit < 64; bbit++)
                if (lo + bbit >= N && ((d[s * words + w] >> bbit) & 1ull)) ok = false;
        }
        if (cnt != (s == 0 ? na : nb)) ok = false;
    }
    if (nv > 2) ok = false;
    unsigned v0 = nv > 0 ? (unsigned)vc[0] : SCQ_NOVIRT, v1 = nv > 1 ? (unsigned)vc[1] : SCQ_NOVIRT;
    keys[i] = key;
    virts[i] = v0 | (v1 << 16);
    valid[i] = ok ? 1 : 0;
}

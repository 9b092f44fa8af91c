// scqmc_setup.hip -- setup kernels: integral blocks over non-core orbitals,
// core folding, and the device tables of the reference wave function
// (determinant -> coefficient; determinant with one / two active electrons
// removed -> the reference determinants it came from).
#include "scqmc_device.h"

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

// table build: expand reference determinants into (key, payload) pairs.
// mode 0: the determinant; 1: one active electron t removed; 2: two, t < u.
// payload = index << 13 | sign << 12 | code, code = t (mode 1) or t<<6|u
// (mode 2); sign = parity of the annihilation string that removes the
// electrons from the determinant: below(t) for one, below(t) + below(u) - 1
// for two (the part of a Slater-Condon phase that depends on the reference
// determinant, folded into the stored coefficient).
__global__ void k_expand(const unsigned long long *rkeys, long long n, int mode, int per, unsigned long long *okeys,
                         unsigned long long *opay) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long k = rkeys[i];
    if (mode == 0) { okeys[i] = k; opay[i] = (unsigned long long)i << 13; return; }
    int codes[64];
    int ne = 0;
    unsigned long long x = k;
    while (x) { int c = __ffsll((long long)x) - 1; x &= x - 1ull; codes[ne++] = c; }
    long long o = i * per;
    if (mode == 1) {
        for (int a = 0; a < ne; a++) {
            unsigned long long sg = (unsigned long long)(key_below(k, codes[a]) & 1);
            okeys[o + a] = k & ~(1ull << codes[a]);
            opay[o + a] = ((unsigned long long)i << 13) | (sg << 12) | (unsigned long long)codes[a];
        }
    } else {
        int m = 0;
        for (int a = 0; a < ne; a++)
            for (int b = a + 1; b < ne; b++) {
                unsigned long long sg = (unsigned long long)((key_below(k, codes[a]) + key_below(k, codes[b]) - 1) & 1);
                okeys[o + m] = k & ~(1ull << codes[a]) & ~(1ull << codes[b]);
                opay[o + m] = ((unsigned long long)i << 13) | (sg << 12) | ((unsigned long long)codes[a] << 6) |
                              (unsigned long long)codes[b];
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

// insert every expanded key into an open-addressing table whose slot keys sit
// at stride `stride` (u64 units); counts entries per slot and distinct keys
__global__ void k_insert(const unsigned long long *ekeys, long long m, unsigned long long *keys, int stride,
                         unsigned long long mask, unsigned *cnt, unsigned *slot_of, unsigned *unique) {
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    unsigned long long key = ekeys[j];
    unsigned long long slot = scq_hash(key) & mask;
    while (true) {
        unsigned long long prev = atomicCAS(&keys[slot * stride], SCQ_EMPTY_KEY, key);
        if (prev == SCQ_EMPTY_KEY) { if (unique) atomicAdd(unique, 1u); break; }
        if (prev == key) break;
        slot = (slot + 1) & mask;
    }
    if (cnt) atomicAdd(&cnt[slot], 1u);
    if (slot_of) slot_of[j] = (unsigned)slot;
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

// sort each list by payload (deterministic content order) and write the
// entries (signed coefficient, code); the determinant table (ents == null)
// keeps the coefficient in the slot instead (one determinant per key)
__global__ void k_finish(const unsigned *cnt, const unsigned *off, long long cap, unsigned long long *tmp,
                         const double *coeff, ulonglong2 *slots, ListEnt *ents) {
    long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    unsigned c = cnt[s], o = off[s];
    if (!ents) {
        slots[s].y = c ? (unsigned long long)__double_as_longlong(coeff[tmp[o] >> 13]) : 0ull;
        return;
    }
    slots[s].y = ((unsigned long long)c << 32) | (unsigned long long)o;
    for (unsigned i = 1; i < c; i++) {
        unsigned long long v = tmp[o + i];
        int j = (int)i - 1;
        while (j >= 0 && tmp[o + j] > v) { tmp[o + j + 1] = tmp[o + j]; j--; }
        tmp[o + j + 1] = v;
    }
    for (unsigned i = 0; i < c; i++) {
        unsigned long long v = tmp[o + i];
        ListEnt e;
        e.val = ((v >> 12) & 1ull) ? -coeff[v >> 13] : coeff[v >> 13];
        e.code = (unsigned)(v & 0xFFFull);
        e.pad = 0u;
        ents[o + i] = e;
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

__global__ void k_fill_slots(ulonglong2 *s, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = make_ulonglong2(SCQ_EMPTY_KEY, 0ull);
}

// FP32 copy of an FP64 array (the precision form's integrals)
__global__ void k_to_f32(const double *in, float *out, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

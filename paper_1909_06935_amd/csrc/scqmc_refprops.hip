// scqmc_refprops.hip -- properties of the reference phi0 used to set up the
// Dyall Hamiltonian of "SC-NEVPT2(s)": its active one-particle density, the
// generalized Fock operator over the virtual orbitals (whose eigenvectors are
// the semicanonical virtuals and whose eigenvalues are the virtual orbital
// energies of H_D), and the rotation of the integrals to those orbitals.
// E_0^(0) = <phi0|H|phi0>/<phi0|phi0> is evaluated with the walker kernel
// restricted to active-space neighbours (k_eval with active_only set).
#include "scqmc_device.h"

// Spin-summed active density, unnormalised, as 128-bit fixed point (fx_add):
// acc[(t*A + u)*2 + {0,1}] += sum_sigma c(d') c(d) <d'|a+_t a_u|d>.
// One thread per reference determinant d; d' = d - u + t looked up in the
// reference table.  Integer atomics keep the sums independent of order.  The
// core electrons below t and u add the same count to both signs (even total).
__global__ void k_ref_rdm1(DevProblem P, const unsigned long long *keys, const double *coef, long long n,
                           unsigned long long *acc) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned long long key = keys[i];
    double cb = coef[i];
    if (cb == 0.0) return;
    int A = P.A;
    uint32_t am = (A >= 32) ? 0xFFFFFFFFu : ((1u << A) - 1u);
    for (int sg = 0; sg < 2; sg++) {
        uint32_t occ = (uint32_t)(key >> (32 * sg)) & am;
        uint32_t o = occ;
        while (o) {
            int u = __ffs(o) - 1;
            o &= o - 1u;
            int cu = 32 * sg + u;
            fx_add(acc + 2 * ((long long)u * A + u), cb * cb);
            unsigned long long k1 = key & ~(1ull << cu);
            int su = key_below(key, cu);
            uint32_t hol = ~occ & am;
            while (hol) {
                int t = __ffs(hol) - 1;
                hol &= hol - 1u;
                int ct = 32 * sg + t;
                unsigned long long k2 = k1 | (1ull << ct);
                double ca = ref_coef(P.ref, k2);
                if (ca == 0.0) continue;
                int e = su + key_below(k1, ct);
                fx_add(acc + 2 * ((long long)t * A + u), (e & 1) ? -ca * cb : ca * cb);
            }
        }
    }
}

// F_ab = h_eff[A+a][A+b] + sum_tu gamma_tu [(ab|tu) - 1/2 (at|ub)] over the
// non-core integral block (h_eff already holds the core terms).
__global__ void k_virtual_fock(DevProblem P, const double *gamma, double *F) {
    int V = P.V, A = P.A;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)V * V) return;
    int a = (int)(i / V), b = (int)(i % V);
    int pa = A + a, pb = A + b;
    double v = P.heff[pa * P.Np + pb];
    for (int t = 0; t < A; t++)
        for (int u = 0; u < A; u++) {
            double g = gamma[t * A + u];
            if (g == 0.0) continue;
            v += g * (eri4(P, pa, pb, t, u) - 0.5 * eri4(P, pa, t, u, pb));
        }
    F[i] = v;
}

// One index of the non-core two-electron block to the rotated virtual basis:
// out[..., x, ...] = in[..., x, ...] for active x, sum_a U[a][b] in[..., A+a, ...]
// for x = A+b (index position pos, 0 = first).
__global__ void k_rotate_eri(const double *in, double *out, int Np, int A, const double *U, int pos) {
    long long tot = (long long)Np * Np * Np * Np;
    long long stride = 1;
    for (int k = pos + 1; k < 4; k++) stride *= Np;
    int V = Np - A;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
        int x = (int)((i / stride) % Np);
        if (x < A) {
            out[i] = in[i];
            continue;
        }
        int b = x - A;
        long long base = i - (long long)x * stride;
        double v = 0.0;
        for (int a = 0; a < V; a++) v += U[a * V + b] * in[base + (long long)(A + a) * stride];
        out[i] = v;
    }
}

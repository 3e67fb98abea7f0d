/* CPU FP64 oracle: matrix-free y = H x for the Hubbard Hamiltonian, Eq. (1).
 *
 * TEST INFRASTRUCTURE ONLY: called by tests/, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 *
 * Plain definition, no tricks:
 *  - basis = tensor product of the per-spin sorted lists of occupation bit
 *    strings (Sec. II.A), composite index r = D_dn * idx_up + idx_dn;
 *  - the diagonal counts doubly occupied sites times U (Sec. II.B);
 *  - each kinetic term amp * c+_a c_b (amp = -t, both directions, both spins)
 *    is applied with explicit operator algebra on the normal-ordered string
 *    (up operators left of down operators, site index increasing right to
 *    left, Sec. II.A), one factor -1 per operator passed;
 *  - the index of every state is found by binary search over the stored
 *    sorted list (the traditional method of Sec. II.C).
 * Row r of y is sum over sources r' of <r|H|r'> x[r']: the sources are the
 * states c+_b c_a |r> of each term, and <r|c+_a c_b|r'> is evaluated by
 * applying the term to |r'>.
 */
#include <stdint.h>

static int popc32(uint32_t v) { return __builtin_popcount(v); }

static int64_t find_sorted(const uint32_t* a, int64_t n, uint32_t key) {
    int64_t lo = 0, hi = n;            /* search [lo, hi) */
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && a[lo] == key) ? lo : -1;
}

/* operators standing left of the slot of site i, spin s, in state (u, d) */
static int ops_left(uint32_t u, uint32_t d, int spin, int i) {
    uint32_t above_u = (i >= 31) ? 0u : (u >> (i + 1));
    uint32_t above_d = (i >= 31) ? 0u : (d >> (i + 1));
    return spin == 0 ? popc32(above_u) : popc32(u) + popc32(above_d);
}

/* apply c+_a c_b (spin s) to (u, d) in place; returns 0 if the result vanishes, else the sign */
static int apply_term(uint32_t* u, uint32_t* d, int spin, int a, int b) {
    uint32_t* s = (spin == 0) ? u : d;
    int count;
    if (!((*s >> b) & 1u)) return 0;
    count = ops_left(*u, *d, spin, b);
    *s &= ~(1u << b);
    if ((*s >> a) & 1u) return 0;
    count += ops_left(*u, *d, spin, a);
    *s |= (1u << a);
    return (count & 1) ? -1 : 1;
}

/* y[r - r0] = (H x)[r] for r in [r0, r1).  Returns 0, or -1 if a state is missing. */
int oracle_hv_rows(int n_bonds, const int32_t* bi, const int32_t* bj, const double* bt, double U,
                   const uint32_t* up, int64_t Dup, const uint32_t* dn, int64_t Ddn,
                   const double* x, double* y, int64_t r0, int64_t r1, int nthreads) {
    int bad = 0;
    int64_t r;
    (void)Dup;
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads) reduction(|:bad)
    for (r = r0; r < r1; r++) {
        int64_t iu = r / Ddn, id = r % Ddn;
        uint32_t pu = up[iu], pd = dn[id];
        double acc = U * (double)popc32(pu & pd) * x[r];
        int k, dir, spin;
        for (k = 0; k < n_bonds; k++) {
            for (dir = 0; dir < 2; dir++) {
                int a = dir ? bj[k] : bi[k];
                int b = dir ? bi[k] : bj[k];
                double amp = -bt[k];
                for (spin = 0; spin < 2; spin++) {
                    uint32_t su = pu, sd = pd, tu, td;
                    int sg;
                    int64_t ju, jd;
                    if (!apply_term(&su, &sd, spin, b, a)) continue;   /* candidate source */
                    tu = su; td = sd;
                    sg = apply_term(&tu, &td, spin, a, b);             /* <r| c+_a c_b |source> */
                    if (sg == 0 || tu != pu || td != pd) { bad = 1; continue; }
                    ju = find_sorted(up, Dup, su);
                    jd = find_sorted(dn, Ddn, sd);
                    if (ju < 0 || jd < 0) { bad = 1; continue; }
                    acc += amp * (double)sg * x[ju * Ddn + jd];
                }
            }
        }
        y[r - r0] = acc;
    }
    return bad ? -1 : 0;
}

/*
 * ORACLE — test infrastructure only.  A stand-alone check of solvers.c, built with gcc's address and
 * undefined-behaviour sanitizers by the CPU test suite (nothing else builds or runs it).
 *
 * On seeded random binary problems F(x) = sum_i un_i x_i + sum_e cap_e |x_a - x_b| (the block problem of Eq. (8)
 * with its weights fixed) of 0 to 12 nodes, it checks the two solvers against brute force written here:
 *   - every labelling's energy from its own loop equals oracle_objective's;
 *   - oracle_enumerate returns the smallest-code minimiser and the minimum energy;
 *   - oracle_mincut (cap_e >= 0 only) returns a minimiser that is contained in every minimiser (the minimal one,
 *     unique for a submodular F), and its flow equals the minimum plus sum_i max(-un_i, 0);
 *   - oracle_mincut refuses a negative capacity with -4.
 * Problems with many ties (small integer unaries and capacities, zeros included) are drawn as often as wide
 * ones.  Prints "ok <problems>" and exits 0, or names the first failing problem and exits 1.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_mincut(int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb, const int64_t *cap,
                  uint8_t *x, int64_t *flow_out);
int oracle_enumerate(int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb, const int64_t *cap,
                     uint8_t *x, int64_t *emin_out);
int64_t oracle_objective(int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb,
                         const int64_t *cap, const uint8_t *x);

/* xorshift64* (Vigna): the check's own problem generator */
static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rng(void) {
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return rng_state * 0x2545F4914F6CDD1Dull;
}
static int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(rng() % (uint64_t)(hi - lo + 1)); }

#define NMAX 12
#define MMAX 40

static int fail(int prob, const char *what) {
    printf("problem %d: %s\n", prob, what);
    return 1;
}

int main(int argc, char **argv) {
    const int n_prob = argc > 1 ? atoi(argv[1]) : 3000;
    int64_t un[NMAX], cap[MMAX];
    int32_t ea[MMAX], eb[MMAX];
    uint8_t x[NMAX], xe[NMAX], xc[NMAX];
    for (int prob = 0; prob < n_prob; ++prob) {
        const int n = (int)uniform(0, NMAX);
        const int m = n >= 2 ? (int)uniform(0, MMAX) : 0;
        const int tie_prone = prob % 2 == 0;
        const int negative = prob % 7 == 3;
        for (int i = 0; i < n; ++i) un[i] = tie_prone ? uniform(-2, 2) : uniform(-1000, 1000);
        for (int e = 0; e < m; ++e) {
            ea[e] = (int32_t)uniform(0, n - 1);
            do { eb[e] = (int32_t)uniform(0, n - 1); } while (eb[e] == ea[e]);
            cap[e] = tie_prone ? uniform(0, 2) : uniform(0, 600);
        }
        if (negative && m > 0) cap[uniform(0, m - 1)] = -uniform(1, 5);
        /* brute force */
        int64_t best = INT64_MAX, src = 0;
        uint32_t best_code = 0;
        for (int i = 0; i < n; ++i) src += un[i] < 0 ? -un[i] : 0;
        for (uint32_t code = 0; code < (1u << n); ++code) {
            int64_t e = 0;
            for (int i = 0; i < n; ++i) {
                x[i] = (uint8_t)((code >> i) & 1u);
                e += x[i] ? un[i] : 0;
            }
            for (int k = 0; k < m; ++k) e += x[ea[k]] != x[eb[k]] ? cap[k] : 0;
            if (oracle_objective(n, un, m, ea, eb, cap, x) != e) return fail(prob, "oracle_objective");
            if (e < best) { best = e; best_code = code; }
        }
        int64_t emin = 0;
        if (oracle_enumerate(n, un, m, ea, eb, cap, xe, &emin) != 0) return fail(prob, "oracle_enumerate rc");
        if (emin != best) return fail(prob, "oracle_enumerate minimum");
        for (int i = 0; i < n; ++i)
            if (xe[i] != ((best_code >> i) & 1u)) return fail(prob, "oracle_enumerate smallest code");
        int64_t flow = 0;
        const int rc = oracle_mincut(n, un, m, ea, eb, cap, xc, &flow);
        int has_negative = 0;
        for (int k = 0; k < m; ++k) has_negative |= cap[k] < 0;
        if (has_negative) {
            if (rc != -4) return fail(prob, "oracle_mincut accepted a negative capacity");
            continue;
        }
        if (rc != 0) return fail(prob, "oracle_mincut rc");
        if (oracle_objective(n, un, m, ea, eb, cap, xc) != best) return fail(prob, "oracle_mincut not a minimiser");
        if (flow != best + src) return fail(prob, "oracle_mincut flow");
        /* contained in every minimiser */
        for (uint32_t code = 0; code < (1u << n); ++code) {
            for (int i = 0; i < n; ++i) x[i] = (uint8_t)((code >> i) & 1u);
            if (oracle_objective(n, un, m, ea, eb, cap, x) != best) continue;
            for (int i = 0; i < n; ++i)
                if (xc[i] && !x[i]) return fail(prob, "oracle_mincut not the minimal minimiser");
        }
    }
    printf("ok %d\n", n_prob);
    return 0;
}

/*
 * metropolis.c -- independent single-spin-flip Metropolis sampler of the 2D
 * classical XY model (paper, Eq. (Hc); periodic L x L square lattice, J = 1).
 *
 * TEST INFRASTRUCTURE ONLY.  It is the second, unrelated Markov chain that the
 * Swendsen-Wang oracle is checked against (both must sample the same Boltzmann
 * distribution).  It shares nothing with xy_oracle.c: it works on angles, uses
 * cos/sin of angle differences for every observable, and draws its numbers from
 * SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), not from Philox.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform double in [0, 1) with 53 random bits */
static double uniform(uint64_t *state) { return (double)(splitmix64(state) >> 11) * 0x1.0p-53; }

/* Local energy of site i's four links for angle th: -sum_nb cos(th - th_nb). */
static double local_energy(const double *th, int64_t L, int64_t x, int64_t y, double t)
{
    double e = 0.0;
    e -= cos(t - th[y * L + (x + 1) % L]);
    e -= cos(t - th[y * L + (x + L - 1) % L]);
    e -= cos(t - th[((y + 1) % L) * L + x]);
    e -= cos(t - th[((y + L - 1) % L) * L + x]);
    return e;
}

/*
 * Runs `nsweeps` Metropolis sweeps (sequential site order, proposal
 * th' = th + delta (2u - 1), acceptance min(1, exp(-beta dE))) after `ntherm`
 * unrecorded sweeps, starting from angles th[N] (updated in place).
 * trace (nsweeps x 5) receives, after each sweep:
 *   E = H / N,  m2 = |sum s / N|^2,  ex = sum_x cos(th_i - th_j) / N,
 *   sx = sum_x sin(th_i - th_j) / N,  ups_x = ex - beta N sx^2
 * where sum_x runs over the links (i, i + x_hat).  Returns the acceptance rate.
 */
double metro_run(int64_t L, double beta, double delta, uint64_t seed, int64_t ntherm,
                 int64_t nsweeps, double *th, double *trace)
{
    uint64_t st = seed;
    int64_t N = L * L;
    int64_t accepted = 0, proposed = 0;
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t sweep = 0; sweep < ntherm + nsweeps; ++sweep) {
        for (int64_t y = 0; y < L; ++y) {
            for (int64_t x = 0; x < L; ++x) {
                int64_t i = y * L + x;
                double old = th[i];
                double prop = old + delta * (2.0 * uniform(&st) - 1.0);
                double dE = local_energy(th, L, x, y, prop) - local_energy(th, L, x, y, old);
                ++proposed;
                if (dE <= 0.0 || uniform(&st) < exp(-beta * dE)) {
                    th[i] = fmod(prop + two_pi, two_pi);
                    ++accepted;
                }
            }
        }
        if (sweep < ntherm) continue;
        double e = 0.0, ex = 0.0, sx = 0.0, mc = 0.0, ms = 0.0;
        for (int64_t y = 0; y < L; ++y) {
            for (int64_t x = 0; x < L; ++x) {
                double t = th[y * L + x];
                double dx = t - th[y * L + (x + 1) % L];
                double dy = t - th[((y + 1) % L) * L + x];
                e -= cos(dx) + cos(dy);
                ex += cos(dx);
                sx += sin(dx);
                mc += cos(t);
                ms += sin(t);
            }
        }
        double n = (double)N;
        double *o = trace + 5 * (sweep - ntherm);
        o[0] = e / n;
        o[1] = (mc * mc + ms * ms) / (n * n);
        o[2] = ex / n;
        o[3] = sx / n;
        o[4] = ex / n - beta * n * (sx / n) * (sx / n);
    }
    return proposed ? (double)accepted / (double)proposed : 0.0;
}

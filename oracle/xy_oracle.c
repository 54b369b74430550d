/*
 * xy_oracle.c -- CPU oracle for the Swendsen-Wang sweep of the 2D classical XY
 * model with Wolff's embedded-cluster formalism, and for the generalized
 * probability-changing-cluster (PCC) beta controller driven by the helicity
 * modulus (Komura & Okabe, arXiv:1210.6116).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct: one thread, FP64
 * arithmetic throughout, breadth-first-search cluster labelling, and its own
 * Philox4x32-10 written from Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11).  It shares no code with the HIP path.
 * Only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load it; the product never does.
 *
 * Model (paper, Eq. (Hc)): H = -J sum_<ij> s_i . s_j on an L x L square
 * lattice with periodic boundary conditions, J = 1, s_i a unit 2-vector.
 * Site index i = y*L + x (x fastest); every site owns two links, (i, right(i))
 * and (i, down(i)), so the lattice has 2N links (at L = 2 each neighbour pair
 * is therefore linked twice, which is what the periodic sum literally gives).
 *
 * Spin storage: the state is a pair of planes (cos, sin).  All arithmetic is
 * FP64; with storage32 != 0 every value written to the state is rounded to
 * FP32 (the lattice is stored in FP32 by the workloads this oracle checks),
 * with storage32 == 0 the state stays FP64.
 *
 * Random-number layout (the interface both implementations follow):
 *   key = (seed mod 2^32, seed div 2^32); u(w) = w * 2^-32 in [0, 1)
 *   BOND ctr = ((y>>1)*L + x, rep, t, 1): words (w0, w1) = (x-link, y-link) of
 *            site (x, y even); words (w2, w3) = same for site (x, y+1)
 *   FLIP ctr = (r>>7, rep, t, 2): the coin of cluster root r is bit (r & 31)
 *            of word ((r >> 5) & 3)
 *   DIR  ctr = (k, rep, t, 3), k = 0, 1, ... attempts of the disk rejection
 *   INIT ctr = (i, rep, k, 4), k = 0, 1, ... attempts of the disk rejection
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAG_BOND 1u
#define TAG_FLIP 2u
#define TAG_DIR 3u
#define TAG_INIT 4u
#define MAX_ATTEMPTS 16
#define RENORM_EVERY 1024u
#define TIE_EPS 1e-9

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): ten rounds of two 32x32->64 multiplications by the */
/* published multipliers, with the key bumped by the Weyl constants between  */
/* rounds.                                                                   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Philox4x64-10, the 64-bit member of the same family (same round shape,    */
/* 64x64->128 products).  It exists only so that the round shape can be      */
/* checked against an independent implementation (numpy's Philox).           */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        uint64_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t w[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

static double unif(uint32_t w) { return (double)w * (1.0 / 4294967296.0); }

static double store(double v, int storage32) { return storage32 ? (double)(float)v : v; }

/* A point uniform on the unit circle, drawn as a point uniform in the unit   */
/* disk (rejection from the square [-1,1]^2) and scaled to unit length.  Used */
/* for the mirror direction of the embedding and for the uniform-angle hot    */
/* start; only correctly rounded operations are involved.  Returns 0 if no   */
/* candidate was accepted within MAX_ATTEMPTS draws (then the point is (1,0)).*/
static int disk_direction(uint64_t seed, uint32_t c1, uint32_t tag, uint32_t idx_word0,
                          uint32_t t_word2, int attempts_in_word0, double *ox, double *oy)
{
    for (uint32_t k = 0; k < MAX_ATTEMPTS; ++k) {
        uint32_t w[4];
        if (attempts_in_word0)
            draw(seed, k, c1, t_word2, tag, w);
        else
            draw(seed, idx_word0, c1, k, tag, w);
        for (int pair = 0; pair < 2; ++pair) {
            double vx = 2.0 * unif(w[2 * pair]) - 1.0;
            double vy = 2.0 * unif(w[2 * pair + 1]) - 1.0;
            double q = vx * vx + vy * vy;
            if (q > 0.0 && q < 1.0) {
                double n = sqrt(q);
                *ox = vx / n;
                *oy = vy / n;
                return 1;
            }
        }
    }
    *ox = 1.0;
    *oy = 0.0;
    return 0;
}

/* Mirror direction r of sweep t (Wolff embedding: one r per sweep). */
void orc_direction(uint64_t seed, uint32_t rep, uint64_t t, double r[2])
{
    disk_direction(seed, rep, TAG_DIR, 0, (uint32_t)t, 1, &r[0], &r[1]);
}

/* Hot start: every angle independent and uniform on [0, 2pi). */
void orc_hot_start(int64_t L, uint64_t seed, uint32_t rep, int storage32, double *c, double *s)
{
    int64_t N = L * L;
    for (int64_t i = 0; i < N; ++i) {
        double x, y;
        disk_direction(seed, rep, TAG_INIT, (uint32_t)i, 0, 0, &x, &y);
        c[i] = store(x, storage32);
        s[i] = store(y, storage32);
    }
}

static int64_t right_of(int64_t i, int64_t L) { return (i / L) * L + (i % L + 1) % L; }
static int64_t down_of(int64_t i, int64_t L) { return ((i / L + 1) % L) * L + i % L; }

/* Bond activation of the embedded Ising model.  With a_i = s_i . r, the link */
/* (i, j) is active with probability p = 1 - exp(min(0, -2 beta a_i a_j)):    */
/* active iff 2 beta a_i a_j > 0 and exp(-2 beta a_i a_j) < 1 - u.            */
/* A decision with |exp(-x) - (1-u)| < 1e-9 is counted as a near tie.        */
static int bond_decision(double ai, double aj, double beta, uint32_t w, int64_t *ties)
{
    double xb = ((2.0 * beta) * ai) * aj;
    double e = (xb > 0.0) ? exp(-xb) : 1.0;
    double one_minus_u = 1.0 - unif(w);
    if (fabs(e - one_minus_u) < TIE_EPS) ++*ties;
    return e < one_minus_u;
}

static double proj(double c, double s, const double r[2]) { return c * r[0] + s * r[1]; }

void orc_bonds(int64_t L, const double *c, const double *s, double beta, const double r[2],
               uint64_t seed, uint32_t rep, uint64_t t, uint8_t *bx, uint8_t *by, int64_t *ties)
{
    int64_t N = L * L;
    *ties = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t x = i % L, y = i / L;
        uint32_t w[4];
        draw(seed, (uint32_t)((y >> 1) * L + x), rep, (uint32_t)t, TAG_BOND, w);
        int half = (int)(y & 1);
        double ai = proj(c[i], s[i], r);
        int64_t jr = right_of(i, L), jd = down_of(i, L);
        bx[i] = (uint8_t)bond_decision(ai, proj(c[jr], s[jr], r), beta, w[2 * half], ties);
        by[i] = (uint8_t)bond_decision(ai, proj(c[jd], s[jd], r), beta, w[2 * half + 1], ties);
    }
}

/* The same decision for n chosen links, given the spins at both ends:      */
/* link k joins site[k] to its right (dir[k] == 0) or lower (dir[k] == 1)    */
/* neighbour; (ci, si) and (cj, sj) are the two end spins.  Used to check a  */
/* lattice too large for a host copy on a sample of its links.              */
void orc_links(int64_t L, int64_t n, const int64_t *site, const uint8_t *dir, const double *ci,
               const double *si, const double *cj, const double *sj, double beta, const double r[2],
               uint64_t seed, uint32_t rep, uint64_t t, uint8_t *active, int64_t *ties)
{
    *ties = 0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t x = site[k] % L, y = site[k] / L;
        uint32_t w[4];
        draw(seed, (uint32_t)((y >> 1) * L + x), rep, (uint32_t)t, TAG_BOND, w);
        uint32_t wk = w[2 * (int)(y & 1) + (dir[k] ? 1 : 0)];
        active[k] = (uint8_t)bond_decision(proj(ci[k], si[k], r), proj(cj[k], sj[k], r), beta, wk, ties);
    }
}

/* Connected components of the active-bond graph by breadth-first search.    */
/* Sites are scanned in ascending index order and each new component is      */
/* labelled by the site that opened it, i.e. by its minimum site index.      */
int orc_label(int64_t L, const uint8_t *bx, const uint8_t *by, int64_t *label)
{
    int64_t N = L * L;
    int64_t *queue = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    if (!queue) return -1;
    for (int64_t i = 0; i < N; ++i) label[i] = -1;
    for (int64_t i = 0; i < N; ++i) {
        if (label[i] >= 0) continue;
        int64_t head = 0, tail = 0;
        label[i] = i;
        queue[tail++] = i;
        while (head < tail) {
            int64_t k = queue[head++];
            int64_t x = k % L, y = k / L;
            int64_t nb[4] = {right_of(k, L), down_of(k, L), y * L + (x + L - 1) % L,
                             ((y + L - 1) % L) * L + x};
            int on[4] = {bx[k], by[k], bx[nb[2]], by[nb[3]]};
            for (int d = 0; d < 4; ++d) {
                if (on[d] && label[nb[d]] < 0) {
                    label[nb[d]] = i;
                    queue[tail++] = nb[d];
                }
            }
        }
    }
    free(queue);
    return 0;
}

/* Coin of the cluster whose canonical root is r: flip with probability 1/2. */
int orc_coin(uint64_t seed, uint32_t rep, uint64_t t, int64_t r)
{
    uint32_t w[4];
    draw(seed, (uint32_t)(r >> 7), rep, (uint32_t)t, TAG_FLIP, w);
    return (int)((w[(r >> 5) & 3] >> (r & 31)) & 1u);
}

/* Reflection of every spin of a flipped cluster in the line perpendicular to */
/* r: s -> s - 2 (s . r) r.                                                    */
void orc_flip(int64_t L, const int64_t *label, double *c, double *s, const double r[2],
              uint64_t seed, uint32_t rep, uint64_t t, int storage32)
{
    int64_t N = L * L;
    for (int64_t i = 0; i < N; ++i) {
        if (!orc_coin(seed, rep, t, label[i])) continue;
        double g = 2.0 * proj(c[i], s[i], r);
        c[i] = store(c[i] - g * r[0], storage32);
        s[i] = store(s[i] - g * r[1], storage32);
    }
}

/* Rescale every spin to unit length (guards the unit-vector constraint     */
/* against accumulated rounding; applied after the flip of every sweep t    */
/* with (t + 1) a multiple of RENORM_EVERY).                                  */
void orc_renorm(int64_t L, double *c, double *s, int storage32)
{
    int64_t N = L * L;
    for (int64_t i = 0; i < N; ++i) {
        double n = sqrt(c[i] * c[i] + s[i] * s[i]);
        c[i] = store(c[i] / n, storage32);
        s[i] = store(s[i] / n, storage32);
    }
}

/* Observables of one configuration (paper: Eq. (Hc), the helicity-modulus  */
/* definitions of e and s over x-links, and <m^2>_L = chi / L^2):            */
/*  obs[0] E  = H / N             obs[1] m2 = |sum_i s_i / N|^2              */
/*  obs[2] ex = sum_x cos / N     obs[3] sx = sum_x sin(th_i - th_j) / N     */
/*  obs[4] ey, obs[5] sy (same over y-links)                                   */
/*  obs[6] ups_x = ex - beta N sx^2 (sample of the helicity modulus)          */
/*  obs[7] mk2 = |sum_r s(r) e^{i k x}|^2 / N^2 at k = 2 pi / L along x: the   */
/*         chi(k) of the second-moment correlation length, over N (as m2 is   */
/*         chi(0) over N); |.|^2 sums the squared moduli of both components  */
void orc_measure(int64_t L, const double *c, const double *s, double beta, double obs[8])
{
    int64_t N = L * L;
    const double pi = 3.14159265358979323846;
    double scx = 0, ssx = 0, scy = 0, ssy = 0, sc = 0, ss = 0;
    double cre = 0, cim = 0, sre = 0, sim = 0; /* Fourier sums of cos and sin planes */
    for (int64_t i = 0; i < N; ++i) {
        int64_t j = right_of(i, L), k = down_of(i, L);
        scx += c[i] * c[j] + s[i] * s[j];
        ssx += s[i] * c[j] - c[i] * s[j];
        scy += c[i] * c[k] + s[i] * s[k];
        ssy += s[i] * c[k] - c[i] * s[k];
        sc += c[i];
        ss += s[i];
        double kx = 2.0 * pi * (double)(i % L) / (double)L;
        cre += c[i] * cos(kx);
        cim += c[i] * sin(kx);
        sre += s[i] * cos(kx);
        sim += s[i] * sin(kx);
    }
    double n = (double)N;
    obs[0] = -(scx + scy) / n;
    obs[1] = (sc * sc + ss * ss) / (n * n);
    obs[2] = scx / n;
    obs[3] = ssx / n;
    obs[4] = scy / n;
    obs[5] = ssy / n;
    obs[6] = obs[2] - beta * n * obs[3] * obs[3];
    obs[7] = (cre * cre + cim * cim + sre * sre + sim * sim) / (n * n);
}

/* One Swendsen-Wang sweep t: direction, bonds, labels, flip, (renormalise), */
/* measure.  Optional outputs (may be NULL): bx, by (N bytes each) and label */
/* (N int64) of this sweep.  Returns 0, or -1 if memory ran out.             */
int orc_sweep(int64_t L, double *c, double *s, double beta, uint64_t seed, uint32_t rep,
              uint64_t t, int storage32, double obs[8], int64_t *ties, uint8_t *bx_out,
              uint8_t *by_out, int64_t *label_out)
{
    int64_t N = L * L;
    uint8_t *bx = bx_out ? bx_out : (uint8_t *)malloc((size_t)N);
    uint8_t *by = by_out ? by_out : (uint8_t *)malloc((size_t)N);
    int64_t *label = label_out ? label_out : (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int rc = 0;
    if (!bx || !by || !label) {
        rc = -1;
        goto done;
    }
    double r[2];
    orc_direction(seed, rep, t, r);
    orc_bonds(L, c, s, beta, r, seed, rep, t, bx, by, ties);
    if (orc_label(L, bx, by, label) != 0) {
        rc = -1;
        goto done;
    }
    orc_flip(L, label, c, s, r, seed, rep, t, storage32);
    if (((t + 1) % RENORM_EVERY) == 0) orc_renorm(L, c, s, storage32);
    orc_measure(L, c, s, beta, obs);
done:
    if (!bx_out) free(bx);
    if (!by_out) free(by);
    if (!label_out) free(label);
    return rc;
}

/* n sweeps from sweep t0 at fixed beta; trace (n x 8, may be NULL) gets the */
/* observables after every sweep, ties (n, may be NULL) the near-tie counts. */
int orc_run(int64_t L, double *c, double *s, double beta, uint64_t seed, uint32_t rep,
            uint64_t t0, int64_t n, int storage32, double *trace, int64_t *ties)
{
    for (int64_t k = 0; k < n; ++k) {
        double obs[8];
        int64_t nt = 0;
        if (orc_sweep(L, c, s, beta, seed, rep, t0 + (uint64_t)k, storage32, obs, &nt, NULL,
                      NULL, NULL) != 0)
            return -1;
        if (trace) memcpy(trace + 8 * k, obs, sizeof obs);
        if (ties) ties[k] = nt;
    }
    return 0;
}

/* Generalized PCC controller (paper: after each measurement window compare  */
/* beta * Upsilon with 0.636508 and move beta by dbeta towards it).  Each     */
/* step runs `window` sweeps at fixed beta; with e and N s^2 averaged over    */
/* the window, beta*Upsilon = beta (<e_x> - beta <N s_x^2>); if it is below   */
/* target beta grows by dbeta, otherwise it shrinks by dbeta.  The step size  */
/* of step k is max(dbeta_min, dbeta0 / 2^(k / halve_every)) (halve_every = 0 */
/* keeps dbeta0).  beta_trace (nsteps, may be NULL) receives beta after each  */
/* step; bu_trace (nsteps, may be NULL) the window's beta*Upsilon.            */
int orc_pcc_run(int64_t L, double *c, double *s, double *beta, uint64_t seed, uint32_t rep,
                uint64_t t0, int64_t nsteps, int64_t window, double dbeta0, double dbeta_min,
                int64_t halve_every, double target, int64_t k0, int storage32,
                double *beta_trace, double *bu_trace)
{
    uint64_t t = t0;
    for (int64_t k = 0; k < nsteps; ++k) {
        double sum_ex = 0.0, sum_ns2 = 0.0;
        for (int64_t w = 0; w < window; ++w) {
            double obs[8];
            int64_t nt = 0;
            if (orc_sweep(L, c, s, *beta, seed, rep, t, storage32, obs, &nt, NULL, NULL, NULL) != 0)
                return -1;
            sum_ex += obs[2];
            sum_ns2 += (double)(L * L) * obs[3] * obs[3];
            ++t;
        }
        double mean_ex = sum_ex / (double)window, mean_ns2 = sum_ns2 / (double)window;
        double bu = *beta * (mean_ex - *beta * mean_ns2);
        double db = dbeta0;
        if (halve_every > 0) {
            int64_t halvings = (k0 + k) / halve_every;
            db = ldexp(dbeta0, -(int)(halvings < 200 ? halvings : 200));
        }
        if (db < dbeta_min) db = dbeta_min;
        *beta += (bu < target) ? db : -db;
        if (beta_trace) beta_trace[k] = *beta;
        if (bu_trace) bu_trace[k] = bu;
    }
    return 0;
}

/* Wrapping of the clusters around the periodic lattice (the observation that */
/* drives the original PCC rule: raise or lower the temperature according to */
/* whether the clusters percolate).  On a torus a cluster percolates when it  */
/* holds a closed path of active links that winds around the lattice: bit 0  */
/* of *wrap is set if some cluster winds along x a nonzero number of times,  */
/* bit 1 if some cluster winds along y.  Breadth-first search from every     */
/* cluster's first site gives each site unwrapped coordinates (a step to the */
/* right neighbour adds 1 to x, to the lower neighbour 1 to y, the reverse   */
/* steps subtract 1); an active link that reaches an already visited site    */
/* with other unwrapped coordinates closes a path whose winding is that      */
/* difference divided by L.  Every link is examined from both ends, so every */
/* fundamental cycle of the search trees is checked.  Returns -1 if memory   */
/* ran out.                                                                   */
int orc_wrap(int64_t L, const uint8_t *bx, const uint8_t *by, int *wrap)
{
    int64_t N = L * L;
    int64_t *queue = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int64_t *ux = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    int64_t *uy = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    uint8_t *seen = (uint8_t *)calloc((size_t)N, 1);
    *wrap = 0;
    if (!queue || !ux || !uy || !seen) {
        free(queue); free(ux); free(uy); free(seen);
        return -1;
    }
    for (int64_t i = 0; i < N; ++i) {
        if (seen[i]) continue;
        int64_t head = 0, tail = 0;
        seen[i] = 1;
        ux[i] = i % L;
        uy[i] = i / L;
        queue[tail++] = i;
        while (head < tail) {
            int64_t k = queue[head++];
            int64_t x = k % L, y = k / L;
            int64_t nb[4] = {right_of(k, L), down_of(k, L), y * L + (x + L - 1) % L,
                             ((y + L - 1) % L) * L + x};
            const int act[4] = {bx[k], by[k], bx[nb[2]], by[nb[3]]};
            int64_t dx[4] = {1, 0, -1, 0}, dy[4] = {0, 1, 0, -1};
            for (int d = 0; d < 4; ++d) {
                if (!act[d]) continue;
                int64_t j = nb[d], ex = ux[k] + dx[d], ey = uy[k] + dy[d];
                if (!seen[j]) {
                    seen[j] = 1;
                    ux[j] = ex;
                    uy[j] = ey;
                    queue[tail++] = j;
                } else {
                    if (ux[j] != ex) *wrap |= 1;
                    if (uy[j] != ey) *wrap |= 2;
                }
            }
        }
    }
    free(queue); free(ux); free(uy); free(seen);
    return 0;
}

/* The original (percolation) PCC rule with the same windows and step sizes */
/* as orc_pcc_run: each step runs `window` sweeps at fixed beta and observes */
/* after every sweep whether some cluster of that sweep wraps around the     */
/* lattice (along x or along y, orc_wrap); P is the fraction of the window's */
/* sweeps in which one did.  If P is below target (e.g. 1/2: the clusters   */
/* percolate less often than not) beta grows by dbeta (the temperature falls */
/* and the links become more likely), otherwise it shrinks by dbeta.         */
/* beta_trace, p_trace (nsteps) and wrap_trace (nsteps * window, the wrap    */
/* bits of every sweep) may be NULL.                                          */
int orc_pcc_perc_run(int64_t L, double *c, double *s, double *beta, uint64_t seed, uint32_t rep,
                     uint64_t t0, int64_t nsteps, int64_t window, double dbeta0, double dbeta_min,
                     int64_t halve_every, double target, int64_t k0, int storage32,
                     double *beta_trace, double *p_trace, int32_t *wrap_trace)
{
    int64_t N = L * L;
    uint8_t *bx = (uint8_t *)malloc((size_t)N), *by = (uint8_t *)malloc((size_t)N);
    if (!bx || !by) {
        free(bx); free(by);
        return -1;
    }
    uint64_t t = t0;
    int rc = 0;
    for (int64_t k = 0; k < nsteps && rc == 0; ++k) {
        int64_t hits = 0;
        for (int64_t w = 0; w < window; ++w) {
            double obs[8];
            int64_t nt = 0;
            int wr = 0;
            if (orc_sweep(L, c, s, *beta, seed, rep, t, storage32, obs, &nt, bx, by, NULL) != 0 ||
                orc_wrap(L, bx, by, &wr) != 0) {
                rc = -1;
                break;
            }
            if (wr) ++hits;
            if (wrap_trace) wrap_trace[k * window + w] = wr;
            ++t;
        }
        if (rc) break;
        double p = (double)hits / (double)window;
        double db = dbeta0;
        if (halve_every > 0) {
            int64_t halvings = (k0 + k) / halve_every;
            db = ldexp(dbeta0, -(int)(halvings < 200 ? halvings : 200));
        }
        if (db < dbeta_min) db = dbeta_min;
        *beta += (p < target) ? db : -db;
        if (beta_trace) beta_trace[k] = *beta;
        if (p_trace) p_trace[k] = p;
    }
    free(bx); free(by);
    return rc;
}

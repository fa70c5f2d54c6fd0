/*
 * hmc_oracle.c -- serial double-precision CPU reference of the parallel
 * adaptive Metropolis sweeps of Lepadatu et al., "Computation of
 * magnetization, exchange stiffness, anisotropy, and susceptibilities in
 * large-scale systems using GPU-accelerated atomistic parallel Monte
 * Carlo algorithms", arXiv:2103.03517.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain loops, no blocking, no fusion; every
 * quantity is computed from its definition so that a reader can check it
 * against the paper by eye.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares
 * no code with the GPU library.
 *
 * What each part follows:
 *   - spin Hamiltonian: Eq. 2 (exchange over the 6 nearest neighbours,
 *     uniaxial and cubic anisotropy, Zeeman);
 *   - acceptance: Eq. 1 with the comparison P < exp(-dE/T) of Table A1;
 *   - red/black ordering and the adaptive cone angle: Sec. 2 and Table A1;
 *   - constrained pair moves with the once-per-sweep M_L: Sec. 2 and
 *     Table A2;
 *   - susceptibility: Eq. 6.
 *
 * Random-number layout (identical by specification on the GPU side, which
 * implements it separately): Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, SC'11) with key (seed low word, seed high word) and counter
 * (sweep, id, tag, instance).  Tags:
 *   0 / 1  standard update of a red / black site, id = site id;
 *   2 / 3  constrained pair move of colour 0 / 1, id = pair index;
 *   4      random initial spin, sweep word 0, id = site id;
 *   5 / 6  Feistel round keys of the colour-0 / colour-1 shuffle, id = 0;
 *   7, 9   random-order serial cross-check (order, update);
 *   8      heat-bath cross-check.
 * Output words: r0 -> cone opening, r1 -> azimuth, r2 -> acceptance.
 * u = (r + 1/2) 2^-32 lies in (0, 1).
 *
 * Readings where the paper is silent (all listed with reasons in the
 * design notes of the repository):
 *   - the cone proposal is uniform in solid angle on the cap of half-angle
 *     theta: cos(alpha) ~ U(cos theta, 1), azimuth ~ U(0, 2 pi), measured in
 *     the orthonormal basis of Duff et al., JCGT 6(1) 2017;
 *   - the proposed spin is renormalised;
 *   - theta is an integer number of degrees in [1, 180]; it grows by one
 *     when the acceptance rate is strictly above 1/2, else shrinks by one;
 *   - Table A2's rotated frame is replaced by projections on e_C, which
 *     gives the same moves for any choice of the frame's y and z axes; a
 *     pair is rejected when the compensating spin has no real solution or
 *     when the new M_L would not be positive;
 *   - the shuffle is a keyed 4-round Feistel permutation with cycle
 *     walking, one per (sweep, colour).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define NCOLS 10  /* history columns: kind, m_l, m_x, m_y, m_z, e, eanis, tau */

struct oracle_lattice {
    int32_t nx, ny, nz;
    int64_t n;
    double J, Ku, eu[3], Kc, h[3];
    uint64_t seed;
    uint32_t instance;
    int32_t apz;        /* z boundary: 0 periodic, 1 anti-periodic, 2 open */
    uint8_t* mask;      /* per-site active-bond bits (x-, x+, y-, y+, z-, z+), or NULL */
    int32_t theta;
    int64_t sweep;
    int64_t accepted_last;
    double* S;
    double* hist;
    int64_t nhist, cap;
};

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon et al. (SC'11).        */
/* ------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   /* multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   /* key increments */
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(const oracle_lattice* L, uint32_t sweep, uint32_t id,
                 uint32_t tag, double u[4], uint32_t r[4])
{
    uint32_t ctr[4] = { sweep, id, tag, L->instance };
    uint32_t key[2] = { (uint32_t)(L->seed & 0xFFFFFFFFu),
                        (uint32_t)(L->seed >> 32) };
    oracle_philox4x32_10(ctr, key, r);
    for (int k = 0; k < 4; ++k)
        u[k] = ((double)r[k] + 0.5) * (1.0 / 4294967296.0);
}

/* ------------------------------------------------------------------ */
/* Shuffle of one colour (Table A2, ShuffleRedBlackSpins).             */
/* ------------------------------------------------------------------ */

/* MurmurHash3 32-bit finaliser (A. Appleby, public domain). */
uint32_t oracle_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* Keyed permutation of [0, n): a balanced 4-round Feistel network on b
 * bits (b the smallest even number >= 2 with 2^b >= n), iterated until the
 * value falls inside [0, n) ("cycle walking"). */
uint32_t oracle_feistel(uint32_t x, uint32_t n, const uint32_t key[4])
{
    int b = 2;
    while (b < 32 && ((uint64_t)1 << b) < (uint64_t)n) b += 2;
    int half = b / 2;
    uint32_t mask = (half >= 32) ? 0xFFFFFFFFu : (((uint32_t)1 << half) - 1u);
    do {
        uint32_t left = x >> half;
        uint32_t right = x & mask;
        for (int round = 0; round < 4; ++round) {
            uint32_t f = oracle_fmix32(right ^ key[round]) & mask;
            uint32_t new_right = left ^ f;
            left = right;
            right = new_right;
        }
        x = (left << half) | right;
    } while (x >= n);
    return x;
}

/* ------------------------------------------------------------------ */
/* Lattice geometry.                                                   */
/* ------------------------------------------------------------------ */

static int64_t site_id(const oracle_lattice* L, int64_t x, int64_t y, int64_t z)
{
    return x + (int64_t)L->nx * (y + (int64_t)L->ny * z);
}

static void coords(const oracle_lattice* L, int64_t i, int64_t* x, int64_t* y,
                   int64_t* z)
{
    *x = i % L->nx;
    *y = (i / L->nx) % L->ny;
    *z = i / ((int64_t)L->nx * L->ny);
}

static int colour_of(const oracle_lattice* L, int64_t i)
{
    int64_t x, y, z;
    coords(L, i, &x, &y, &z);
    return (int)((x + y + z) & 1);
}

/* The idx-th site of colour c, counting sites of that colour in increasing
 * site id.  Because nx is even, every aligned pair of ids (2a, 2a+1) holds
 * exactly one site of each colour. */
int64_t oracle_site_of(const oracle_lattice* L, int32_t colour, int64_t idx)
{
    int64_t s = 2 * idx;
    if (colour_of(L, s) != colour) s += 1;
    return s;
}

/* Neighbours of site i in the order x-, x+, y-, y+, z-, z+ (periodic
 * indexing), and the weight each one enters the exchange with: -1 for a bond
 * that crosses the z boundary of an anti-periodic lattice, 0 for one that
 * crosses an open z boundary or whose bit is clear in the site's bond mask,
 * else +1. */
static void neighbours(const oracle_lattice* L, int64_t i, int64_t nb[6], double sg[6])
{
    int64_t x, y, z;
    coords(L, i, &x, &y, &z);
    nb[0] = site_id(L, (x - 1 + L->nx) % L->nx, y, z);
    nb[1] = site_id(L, (x + 1) % L->nx, y, z);
    nb[2] = site_id(L, x, (y - 1 + L->ny) % L->ny, z);
    nb[3] = site_id(L, x, (y + 1) % L->ny, z);
    nb[4] = site_id(L, x, y, (z - 1 + L->nz) % L->nz);
    nb[5] = site_id(L, x, y, (z + 1) % L->nz);
    for (int k = 0; k < 6; ++k) sg[k] = 1.0;
    if (L->apz) {
        const double w = L->apz == 1 ? -1.0 : 0.0;
        if (z == 0) sg[4] = w;
        if (z == L->nz - 1) sg[5] = w;
    }
    if (L->mask)
        for (int k = 0; k < 6; ++k)
            if (!((L->mask[i] >> k) & 1u)) sg[k] = 0.0;
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ------------------------------------------------------------------ */
/* Energies (Eq. 2).                                                   */
/* ------------------------------------------------------------------ */

static double cubic_f(const double s[3])
{
    double x2 = s[0] * s[0], y2 = s[1] * s[1], z2 = s[2] * s[2];
    return x2 * y2 + x2 * z2 + y2 * z2;
}

/* E_i of Eq. 2 for site i holding the direction S, the other spins fixed. */
double oracle_local_energy(const oracle_lattice* L, int64_t i, const double S[3])
{
    int64_t nb[6];
    double sg[6];
    neighbours(L, i, nb, sg);
    double exch = 0.0;
    for (int k = 0; k < 6; ++k) exch += sg[k] * dot3(S, &L->S[3 * nb[k]]);
    double se = dot3(S, L->eu);
    return -L->J * exch - L->Ku * se * se + L->Kc * cubic_f(S) - dot3(L->h, S);
}

/* Total energy: the Hamiltonian whose site terms are Eq. 2, with every
 * exchange bond counted once (bond i -> i+x, i+y, i+z). */
static void energy_parts(const oracle_lattice* L, double* e_exch, double* e_uni,
                         double* e_cub, double* e_zee)
{
    double ex = 0.0, eu = 0.0, ec = 0.0, ez = 0.0;
    for (int64_t i = 0; i < L->n; ++i) {
        int64_t nb[6];
        double sg[6];
        neighbours(L, i, nb, sg);
        const double* s = &L->S[3 * i];
        ex += -L->J * (sg[1] * dot3(s, &L->S[3 * nb[1]]) + sg[3] * dot3(s, &L->S[3 * nb[3]]) +
                       sg[5] * dot3(s, &L->S[3 * nb[5]]));
        double se = dot3(s, L->eu);
        eu += -L->Ku * se * se;
        ec += L->Kc * cubic_f(s);
        ez += -dot3(L->h, s);
    }
    *e_exch = ex; *e_uni = eu; *e_cub = ec; *e_zee = ez;
}

double oracle_total_energy(const oracle_lattice* L)
{
    double a, b, c, d;
    energy_parts(L, &a, &b, &c, &d);
    return a + b + c + d;
}

/* Torque of the anisotropy field: sum_i S_i x (-dE_anis/dS_i), with
 * E_anis = -Ku (S.e)^2 + Kc f(S). */
static void anis_torque(const oracle_lattice* L, double tau[3])
{
    tau[0] = tau[1] = tau[2] = 0.0;
    for (int64_t i = 0; i < L->n; ++i) {
        const double* s = &L->S[3 * i];
        double se = dot3(s, L->eu);
        double g[3];  /* -dE_anis/dS */
        g[0] = 2.0 * L->Ku * se * L->eu[0] - L->Kc * 2.0 * s[0] * (s[1] * s[1] + s[2] * s[2]);
        g[1] = 2.0 * L->Ku * se * L->eu[1] - L->Kc * 2.0 * s[1] * (s[0] * s[0] + s[2] * s[2]);
        g[2] = 2.0 * L->Ku * se * L->eu[2] - L->Kc * 2.0 * s[2] * (s[0] * s[0] + s[1] * s[1]);
        tau[0] += s[1] * g[2] - s[2] * g[1];
        tau[1] += s[2] * g[0] - s[0] * g[2];
        tau[2] += s[0] * g[1] - s[1] * g[0];
    }
}

/* ------------------------------------------------------------------ */
/* Cone proposal (Table A1, UniformRandom_RotateSpin).                 */
/* ------------------------------------------------------------------ */

/* Orthonormal basis (b1, b2) perpendicular to the unit vector n: the
 * branchless construction of Duff et al., JCGT 6(1), 2017. */
void oracle_onb(const double n[3], double b1[3], double b2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a;
    b1[1] = sign * b;
    b1[2] = -sign * n[0];
    b2[0] = b;
    b2[1] = sign + n[1] * n[1] * a;
    b2[2] = -n[1];
}

/* 1 - cos(theta), written as 2 sin^2(theta/2) for accuracy at small theta. */
static double cone_c1(int theta_deg)
{
    double s = sin((double)theta_deg * M_PI / 360.0);
    return 2.0 * s * s;
}

static void cone_move_c1(const double S[3], double u0, double u1, double c1,
                         double out[3])
{
    double d = u0 * c1;                    /* 1 - cos(alpha), uniform */
    double cosa = 1.0 - d;
    double sina = sqrt(d * (2.0 - d));
    double phi = 2.0 * M_PI * u1;
    double b1[3], b2[3];
    oracle_onb(S, b1, b2);
    double cp = cos(phi), sp = sin(phi);
    double v[3];
    for (int a = 0; a < 3; ++a)
        v[a] = cosa * S[a] + sina * (cp * b1[a] + sp * b2[a]);
    double len = sqrt(dot3(v, v));
    for (int a = 0; a < 3; ++a) out[a] = v[a] / len;
}

void oracle_cone_move(const double S[3], double u0, double u1,
                      int32_t theta_deg, double out[3])
{
    cone_move_c1(S, u0, u1, cone_c1(theta_deg), out);
}

/* Adaptive cone angle of Table A1: one degree up when the acceptance rate
 * (accepted / N) is strictly above 1/2, else one degree down, kept in
 * [1, 180]. */
static void adapt_theta(oracle_lattice* L, int64_t accepted)
{
    double rate = (double)accepted / (double)L->n;
    if (rate > 0.5) {
        if (L->theta < 180) L->theta += 1;
    } else {
        if (L->theta > 1) L->theta -= 1;
    }
}

/* ------------------------------------------------------------------ */
/* Construction and state.                                             */
/* ------------------------------------------------------------------ */

oracle_lattice* oracle_create(int32_t nx, int32_t ny, int32_t nz,
                              double J, double Ku, const double eu[3],
                              double Kc, const double h[3],
                              uint64_t seed, uint32_t instance,
                              int32_t theta0_deg)
{
    /* an odd nz is only meaningful with the open z boundary (set after
     * creation); the sweeps refuse it otherwise */
    if (nx < 2 || ny < 2 || nz < 1 || (nx & 1) || (ny & 1))
        return NULL;
    oracle_lattice* L = (oracle_lattice*)calloc(1, sizeof(oracle_lattice));
    if (!L) return NULL;
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->n = (int64_t)nx * ny * nz;
    L->J = J; L->Ku = Ku; L->Kc = Kc;
    double len = sqrt(dot3(eu, eu));
    for (int a = 0; a < 3; ++a) {
        L->eu[a] = (len > 0.0) ? eu[a] / len : 0.0;
        L->h[a] = h[a];
    }
    L->seed = seed;
    L->instance = instance;
    L->theta = theta0_deg;
    L->S = (double*)calloc((size_t)(3 * L->n), sizeof(double));
    if (!L->S) { free(L); return NULL; }
    return L;
}

void oracle_set_boundary_z(oracle_lattice* L, int32_t mode)
{
    L->apz = (mode == 1 || mode == 2) ? mode : 0;
}

int oracle_set_bond_masks(oracle_lattice* L, const uint8_t* mask)
{
    if (!mask) {
        free(L->mask);
        L->mask = NULL;
        return 0;
    }
    if (!L->mask) L->mask = (uint8_t*)malloc((size_t)L->n);
    if (!L->mask) return -1;
    memcpy(L->mask, mask, (size_t)L->n);
    return 0;
}

/* A checkerboard pass needs a bipartite lattice: an odd periodic nz is not. */
static int sweepable(const oracle_lattice* L)
{
    return !((L->nz & 1) && L->apz != 2);
}

void oracle_destroy(oracle_lattice* L)
{
    if (!L) return;
    free(L->S);
    free(L->hist);
    free(L->mask);
    free(L);
}

void oracle_init_aligned(oracle_lattice* L, const double dir[3])
{
    double len = sqrt(dot3(dir, dir));
    for (int64_t i = 0; i < L->n; ++i)
        for (int a = 0; a < 3; ++a) L->S[3 * i + a] = dir[a] / len;
}

/* Uniform on the sphere: z = 2 u0 - 1, azimuth 2 pi u1. */
void oracle_init_random(oracle_lattice* L)
{
    for (int64_t i = 0; i < L->n; ++i) {
        double u[4];
        uint32_t r[4];
        draw(L, 0u, (uint32_t)i, 4u, u, r);
        double z = 2.0 * u[0] - 1.0;
        double rho = sqrt(1.0 - z * z);
        double phi = 2.0 * M_PI * u[1];
        L->S[3 * i + 0] = rho * cos(phi);
        L->S[3 * i + 1] = rho * sin(phi);
        L->S[3 * i + 2] = z;
    }
}

void oracle_set_spins(oracle_lattice* L, const double* S)
{
    memcpy(L->S, S, (size_t)(3 * L->n) * sizeof(double));
}

void oracle_get_spins(const oracle_lattice* L, double* S)
{
    memcpy(S, L->S, (size_t)(3 * L->n) * sizeof(double));
}

void oracle_get_counters(const oracle_lattice* L, int32_t* theta_deg,
                         int64_t* sweeps_done)
{
    *theta_deg = L->theta;
    *sweeps_done = L->sweep;
}

void oracle_set_counters(oracle_lattice* L, int32_t theta_deg, int64_t sweeps_done)
{
    L->theta = theta_deg;
    L->sweep = sweeps_done;
}

/* ------------------------------------------------------------------ */
/* Sampling.                                                           */
/* ------------------------------------------------------------------ */

static void record_sample(oracle_lattice* L, int constrained)
{
    if (L->nhist == L->cap) {
        int64_t cap = L->cap ? 2 * L->cap : 1024;
        double* p = (double*)realloc(L->hist, (size_t)(cap * NCOLS) * sizeof(double));
        if (!p) return;
        L->hist = p;
        L->cap = cap;
    }
    double M[3] = { 0.0, 0.0, 0.0 };
    for (int64_t i = 0; i < L->n; ++i)
        for (int a = 0; a < 3; ++a) M[a] += L->S[3 * i + a];
    double ex, eu, ec, ez, tau[3];
    energy_parts(L, &ex, &eu, &ec, &ez);
    anis_torque(L, tau);
    double N = (double)L->n;
    double* row = &L->hist[L->nhist * NCOLS];
    row[0] = constrained ? 1.0 : 0.0;
    row[1] = sqrt(dot3(M, M)) / N;
    row[2] = M[0] / N;
    row[3] = M[1] / N;
    row[4] = M[2] / N;
    row[5] = (ex + eu + ec + ez) / N;
    row[6] = (eu + ec) / N;
    row[7] = tau[0] / N;
    row[8] = tau[1] / N;
    row[9] = tau[2] / N;
    L->nhist += 1;
}

void oracle_reset_stats(oracle_lattice* L)
{
    L->nhist = 0;
}

int64_t oracle_samples(const oracle_lattice* L, double* out, int64_t max_rows)
{
    int64_t rows = L->nhist < max_rows ? L->nhist : max_rows;
    for (int64_t r = 0; r < rows; ++r)
        for (int c = 1; c < NCOLS; ++c)
            out[r * (NCOLS - 1) + (c - 1)] = L->hist[r * NCOLS + c];
    return rows;
}

void oracle_observables(const oracle_lattice* L, double T, oracle_obs* o)
{
    memset(o, 0, sizeof(*o));
    o->n = L->n;
    o->sweeps_done = L->sweep;
    o->samples = L->nhist;
    o->accepted_last = L->accepted_last;
    o->theta_deg = L->theta;
    for (int64_t i = 0; i < L->n; ++i)
        for (int a = 0; a < 3; ++a) o->M[a] += L->S[3 * i + a];
    o->m = sqrt(dot3(o->M, o->M)) / (double)L->n;
    energy_parts(L, &o->E_exch, &o->E_uni, &o->E_cub, &o->E_zee);
    o->E = o->E_exch + o->E_uni + o->E_cub + o->E_zee;
    anis_torque(L, o->torque);

    int64_t ns = L->nhist;
    if (ns == 0) return;
    for (int c = 0; c < 4; ++c) {
        double mean = 0.0;
        for (int64_t r = 0; r < ns; ++r) mean += L->hist[r * NCOLS + 1 + c];
        mean /= (double)ns;
        double var = 0.0;
        for (int64_t r = 0; r < ns; ++r) {
            double d = L->hist[r * NCOLS + 1 + c] - mean;
            var += d * d;
        }
        var /= (double)ns;
        o->mean_m[c] = mean;
        o->var_m[c] = var;
        o->chi[c] = (double)L->n * var / T;            /* Eq. 6, mu_S = k_B = 1 */
    }
    double mean = 0.0, var = 0.0, mean_an = 0.0;
    for (int64_t r = 0; r < ns; ++r) {
        mean += L->hist[r * NCOLS + 5];
        mean_an += L->hist[r * NCOLS + 6];
    }
    mean /= (double)ns;
    mean_an /= (double)ns;
    for (int64_t r = 0; r < ns; ++r) {
        double d = L->hist[r * NCOLS + 5] - mean;
        var += d * d;
    }
    o->mean_E = mean;
    o->var_E = var / (double)ns;
    o->mean_Eanis = mean_an;
    int64_t nc = 0;
    for (int64_t r = 0; r < ns; ++r) {
        if (L->hist[r * NCOLS] == 0.0) continue;
        nc += 1;
        for (int a = 0; a < 3; ++a) o->mean_torque[a] += L->hist[r * NCOLS + 7 + a];
    }
    if (nc > 0)
        for (int a = 0; a < 3; ++a) o->mean_torque[a] /= (double)nc;
}

/* ------------------------------------------------------------------ */
/* Standard sweep (Table A1).                                          */
/* ------------------------------------------------------------------ */

/* One attempted update of site i with the random words u (Eq. 1, Eq. 2). */
static int metropolis_site(oracle_lattice* L, int64_t i, const double u[4],
                           double c1, double T)
{
    double* s = &L->S[3 * i];
    double trial[3];
    cone_move_c1(s, u[0], u[1], c1, trial);
    double dE = oracle_local_energy(L, i, trial) - oracle_local_energy(L, i, s);
    double P = u[2];
    if (P < exp(-dE / T)) {
        s[0] = trial[0]; s[1] = trial[1]; s[2] = trial[2];
        return 1;
    }
    return 0;
}

int64_t oracle_sweep(oracle_lattice* L, double T, int32_t n_sweeps, int32_t sample)
{
    if (!sweepable(L)) return -1;
    for (int32_t it = 0; it < n_sweeps; ++it) {
        int64_t accepted = 0;
        double c1 = cone_c1(L->theta);
        for (int colour = 0; colour < 2; ++colour) {        /* red, then black */
            for (int64_t i = 0; i < L->n; ++i) {
                if (colour_of(L, i) != colour) continue;
                double u[4];
                uint32_t r[4];
                draw(L, (uint32_t)L->sweep, (uint32_t)i, (uint32_t)colour, u, r);
                accepted += metropolis_site(L, i, u, c1, T);
            }
        }
        adapt_theta(L, accepted);
        L->accepted_last = accepted;
        L->sweep += 1;
        if (sample) record_sample(L, 0);
    }
    return L->accepted_last;
}

/* ------------------------------------------------------------------ */
/* Constrained sweep (Table A2).                                       */
/* ------------------------------------------------------------------ */

int64_t oracle_constrained_sweep(oracle_lattice* L, double T, const double eC_in[3],
                                 int32_t n_sweeps, int32_t sample,
                                 int32_t exact_serial)
{
    if (!sweepable(L)) return -1;
    double len = sqrt(dot3(eC_in, eC_in));
    double eC[3] = { eC_in[0] / len, eC_in[1] / len, eC_in[2] / len };
    int64_t Nc = L->n / 2;
    for (int32_t it = 0; it < n_sweeps; ++it) {
        /* Magnetisation length along e_C, once at the start of the sweep. */
        double ML = 0.0;
        for (int64_t i = 0; i < L->n; ++i) ML += dot3(&L->S[3 * i], eC);
        double c1 = cone_c1(L->theta);
        int64_t accepted = 0;
        for (int colour = 0; colour < 2; ++colour) {
            uint32_t key[4], rk[4];
            double uk[4];
            draw(L, (uint32_t)L->sweep, 0u, (uint32_t)(5 + colour), uk, rk);
            for (int a = 0; a < 4; ++a) key[a] = rk[a];
            for (int64_t k = 0; k < Nc / 2; ++k) {
                int64_t ia = oracle_feistel((uint32_t)(2 * k), (uint32_t)Nc, key);
                int64_t ja = oracle_feistel((uint32_t)(2 * k + 1), (uint32_t)Nc, key);
                int64_t i = oracle_site_of(L, colour, ia);
                int64_t j = oracle_site_of(L, colour, ja);
                double u[4];
                uint32_t r[4];
                draw(L, (uint32_t)L->sweep, (uint32_t)k, (uint32_t)(2 + colour), u, r);

                double* si = &L->S[3 * i];
                double* sj = &L->S[3 * j];
                double si_new[3], sj_new[3];
                cone_move_c1(si, u[0], u[1], c1, si_new);

                /* components along e_C and perpendicular to it */
                double pi_old = dot3(si, eC), pi_new = dot3(si_new, eC);
                double pj_old = dot3(sj, eC);
                double perp_j_new[3];
                for (int a = 0; a < 3; ++a) {
                    double perp_i_old = si[a] - pi_old * eC[a];
                    double perp_i_new = si_new[a] - pi_new * eC[a];
                    double perp_j_old = sj[a] - pj_old * eC[a];
                    perp_j_new[a] = perp_j_old + perp_i_old - perp_i_new;
                }
                double q = dot3(sj, sj) - dot3(perp_j_new, perp_j_new);
                if (!(q > 0.0)) continue;                      /* no real solution */
                double pj_new = (pj_old >= 0.0 ? 1.0 : -1.0) * sqrt(q);
                for (int a = 0; a < 3; ++a) sj_new[a] = perp_j_new[a] + pj_new * eC[a];

                double Mhat = fabs(ML) + pi_new + pj_new - pi_old - pj_old;
                if (!(Mhat > 0.0) || ML == 0.0) continue;

                double dE = oracle_local_energy(L, i, si_new) - oracle_local_energy(L, i, si)
                          + oracle_local_energy(L, j, sj_new) - oracle_local_energy(L, j, sj);
                double ratio = (Mhat / ML) * (Mhat / ML) * fabs(pj_old / pj_new);
                double P = u[2];
                if (P < ratio * exp(-dE / T)) {
                    for (int a = 0; a < 3; ++a) { si[a] = si_new[a]; sj[a] = sj_new[a]; }
                    accepted += 2;
                    if (exact_serial) ML = (ML > 0.0 ? Mhat : -Mhat);
                }
            }
        }
        adapt_theta(L, accepted);
        L->accepted_last = accepted;
        L->sweep += 1;
        if (sample) record_sample(L, 1);
    }
    return L->accepted_last;
}

/* ------------------------------------------------------------------ */
/* Cross-check samplers (not part of the parallel method).             */
/* ------------------------------------------------------------------ */

int64_t oracle_serial_random_sweep(oracle_lattice* L, double T, int32_t n_sweeps,
                                   int32_t sample)
{
    if (!sweepable(L)) return -1;
    int64_t* order = (int64_t*)malloc((size_t)L->n * sizeof(int64_t));
    if (!order) return -1;
    for (int32_t it = 0; it < n_sweeps; ++it) {
        for (int64_t i = 0; i < L->n; ++i) order[i] = i;
        /* Fisher-Yates shuffle of the site order */
        for (int64_t t = 0; t + 1 < L->n; ++t) {
            double u[4];
            uint32_t r[4];
            draw(L, (uint32_t)L->sweep, (uint32_t)t, 7u, u, r);
            int64_t j = t + (int64_t)(u[0] * (double)(L->n - t));
            if (j >= L->n) j = L->n - 1;
            int64_t tmp = order[t]; order[t] = order[j]; order[j] = tmp;
        }
        double c1 = cone_c1(L->theta);
        int64_t accepted = 0;
        for (int64_t t = 0; t < L->n; ++t) {
            double u[4];
            uint32_t r[4];
            draw(L, (uint32_t)L->sweep, (uint32_t)t, 9u, u, r);
            accepted += metropolis_site(L, order[t], u, c1, T);
        }
        adapt_theta(L, accepted);
        L->accepted_last = accepted;
        L->sweep += 1;
        if (sample) record_sample(L, 0);
    }
    free(order);
    return L->accepted_last;
}

/* Exact conditional sampling of a spin in the local field h_loc: the density
 * is proportional to exp(h_loc . S / T), so w = cos(angle to h_loc) has
 * density proportional to exp(k w) on [-1, 1], k = |h_loc| / T, sampled by
 * inverting its distribution function. */
void oracle_heatbath_sweep(oracle_lattice* L, double T, int32_t n_sweeps, int32_t sample)
{
    if (!sweepable(L)) return;
    for (int32_t it = 0; it < n_sweeps; ++it) {
        for (int64_t i = 0; i < L->n; ++i) {
            int64_t nb[6];
            double sg[6];
            neighbours(L, i, nb, sg);
            double hl[3] = { L->h[0], L->h[1], L->h[2] };
            for (int k = 0; k < 6; ++k)
                for (int a = 0; a < 3; ++a) hl[a] += L->J * sg[k] * L->S[3 * nb[k] + a];
            double hn = sqrt(dot3(hl, hl));
            double u[4];
            uint32_t r[4];
            draw(L, (uint32_t)L->sweep, (uint32_t)i, 8u, u, r);
            double k = hn / T;
            double w;
            if (k < 1e-12) w = 2.0 * u[0] - 1.0;
            else w = 1.0 + log(u[0] + (1.0 - u[0]) * exp(-2.0 * k)) / k;
            if (w > 1.0) w = 1.0;
            if (w < -1.0) w = -1.0;
            double axis[3] = { 0.0, 0.0, 1.0 };
            if (hn > 0.0) for (int a = 0; a < 3; ++a) axis[a] = hl[a] / hn;
            double b1[3], b2[3];
            oracle_onb(axis, b1, b2);
            double phi = 2.0 * M_PI * u[1];
            double st = sqrt(1.0 - w * w);
            for (int a = 0; a < 3; ++a)
                L->S[3 * i + a] = w * axis[a] + st * (cos(phi) * b1[a] + sin(phi) * b2[a]);
        }
        L->sweep += 1;
        if (sample) record_sample(L, 0);
    }
}

/*
 * oracle.h -- serial double-precision CPU reference of the parallel
 * Metropolis sweeps of Lepadatu et al., arXiv:2103.03517.
 *
 * TEST INFRASTRUCTURE ONLY.  This reference exists so that the GPU
 * library can be checked against something plain and slow.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant generator
 * with the HIP library under paper_2103_03517_amd/.
 *
 * Conventions (reduced units: J is the energy unit, k_B = 1, the
 * moment mu_S is folded into the field h):
 *   - site id i = x + nx*(y + ny*z), spins stored as S[3*i + a] (AoS);
 *   - colour of a site is (x + y + z) & 1, red = 0 is updated first
 *     (Sec. 2 and Table A1);
 *   - random numbers: Philox4x32-10 with key = (seed lo, seed hi) and
 *     counter = (sweep, id, tag, instance); the tags are listed in
 *     hmc_oracle.c.
 */
#ifndef HMC_ORACLE_H
#define HMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_lattice oracle_lattice;

/* Averages over the sampled sweeps, each computed from the stored
 * per-sweep samples by its plain definition (mean, then the mean of the
 * squared deviations).  alpha index: 0 = l (length), 1 = x, 2 = y, 3 = z. */
typedef struct {
    int64_t n;                 /* number of spins */
    int64_t sweeps_done;       /* global sweep counter */
    int64_t samples;           /* sampled sweeps since the last reset */
    int64_t accepted_last;     /* accepted single-site updates in the last sweep
                                  (a constrained pair counts 2) */
    int32_t theta_deg;         /* current cone angle, degrees */
    double  M[3];              /* instantaneous total moment sum_i S_i */
    double  m;                 /* |M| / N */
    double  E;                 /* instantaneous total energy, bonds counted once */
    double  E_exch, E_uni, E_cub, E_zee;
    double  torque[3];         /* sum_i S_i x (-dE_anis/dS_i) */
    double  mean_m[4];         /* <m_alpha> */
    double  var_m[4];          /* <m_alpha^2> - <m_alpha>^2 */
    double  mean_E;            /* <E>/N */
    double  var_E;             /* variance of E/N */
    double  mean_Eanis;        /* <E_uni + E_cub>/N */
    double  mean_torque[3];    /* <torque>/N */
    double  chi[4];            /* N var(m_alpha) / T, Eq. 6 in reduced units */
} oracle_obs;

oracle_lattice* oracle_create(int32_t nx, int32_t ny, int32_t nz,
                              double J, double Ku, const double eu[3],
                              double Kc, const double h[3],
                              uint64_t seed, uint32_t instance,
                              int32_t theta0_deg);
void    oracle_destroy(oracle_lattice* L);

/* Initial states. */
/* Boundary along z: 0 periodic (the default), 1 anti-periodic (the bond
 * between planes nz-1 and 0 enters the exchange with a minus sign; the
 * domain-wall method of Sec. 3), 2 open (no bond across the z boundary: a
 * film, Sec. 4).  An odd nz is accepted by oracle_create for the open
 * boundary only: the sweeps return -1 for an odd nz that is not open. */
void    oracle_set_boundary_z(oracle_lattice* L, int32_t mode);
/* Per-site bond masks (N bytes in site order; bit k set = bond k active, in
 * the neighbour order x-, x+, y-, y+, z-, z+), copied; NULL restores every
 * bond.  A bond must be set or clear in both of its sites.  Used for
 * granular films, whose bonds between grains carry no exchange (Sec. 4). */
int     oracle_set_bond_masks(oracle_lattice* L, const uint8_t* mask);
void    oracle_init_aligned(oracle_lattice* L, const double dir[3]);
void    oracle_init_random(oracle_lattice* L);
void    oracle_set_spins(oracle_lattice* L, const double* S);
void    oracle_get_spins(const oracle_lattice* L, double* S);

/* Cone angle and sweep counter (part of the chain state). */
void    oracle_get_counters(const oracle_lattice* L, int32_t* theta_deg,
                            int64_t* sweeps_done);
void    oracle_set_counters(oracle_lattice* L, int32_t theta_deg,
                            int64_t sweeps_done);

/* Standard checkerboard sweeps (Table A1).  If sample != 0 every sweep is
 * recorded.  Returns the accepted updates of the last sweep. */
int64_t oracle_sweep(oracle_lattice* L, double T, int32_t n_sweeps,
                     int32_t sample);

/* Constrained pair sweeps (Table A2).  exact_serial != 0 selects the serial
 * variant in which M_L follows every accepted pair instead of being taken
 * once per sweep; it exists only as a statistical cross-check. */
int64_t oracle_constrained_sweep(oracle_lattice* L, double T,
                                 const double eC[3], int32_t n_sweeps,
                                 int32_t sample, int32_t exact_serial);

/* Serial single-site Metropolis in a random site order (the serial
 * algorithm of Sec. 2).  Cross-check only. */
int64_t oracle_serial_random_sweep(oracle_lattice* L, double T,
                                   int32_t n_sweeps, int32_t sample);

/* Heat-bath sweep: every site is redrawn from its exact conditional
 * distribution.  Valid only with Ku = Kc = 0.  Cross-check only. */
void    oracle_heatbath_sweep(oracle_lattice* L, double T, int32_t n_sweeps,
                              int32_t sample);

void    oracle_reset_stats(oracle_lattice* L);
void    oracle_observables(const oracle_lattice* L, double T, oracle_obs* out);
/* Per-sample history: rows of (m_l, m_x, m_y, m_z, E/N, Eanis/N,
 * tau_x/N, tau_y/N, tau_z/N).  Returns the number of rows copied. */
int64_t oracle_samples(const oracle_lattice* L, double* out, int64_t max_rows);

/* Pieces of the method, exposed for the pin tests. */
void     oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                              uint32_t out[4]);
uint32_t oracle_fmix32(uint32_t h);
uint32_t oracle_feistel(uint32_t x, uint32_t n, const uint32_t key[4]);
void     oracle_onb(const double n[3], double b1[3], double b2[3]);
void     oracle_cone_move(const double S[3], double u0, double u1,
                          int32_t theta_deg, double out[3]);
double   oracle_local_energy(const oracle_lattice* L, int64_t site,
                             const double S[3]);
double   oracle_total_energy(const oracle_lattice* L);
int64_t  oracle_site_of(const oracle_lattice* L, int32_t colour, int64_t idx);

#ifdef __cplusplus
}
#endif
#endif

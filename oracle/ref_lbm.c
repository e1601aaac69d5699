/*
 * Plain scalar FP64 reference of the D3Q19 LBM-MRT-Smagorinsky-Guo update.
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
 * baseline of the benchmark load this library.  It shares no code, header or
 * table with the HIP path; every constant below is typed in from the paper.
 *
 * Method (one time step, every cell, in the paper's order):
 *   rho = sum f, rho u = sum f c + F/2               App. A eq. guo_velocity
 *   m = M f                                          App. B eq. moment-matrix
 *   m_eq, F_m                                        App. B eq. meq_fm
 *   S_ab from m_neq = m - m_eq                       App. B.1 eq. yu_strain
 *   |S| = sqrt(2 S:S)                                Sec. 2.3 eq. strain_norm
 *   tau_e = 1/2 + 3 (nu0 + C Delta^2 |S|)            Sec. 2.3 eq. les_viscosity
 *   m* = m - Lambda m_neq + (I - Lambda/2) F_m       Sec. 2.3 eq. mrt_les_guo
 *   f* = M^-1 m*,  f(x + c, t+1) = f*(x, t)          App. A eq. mrt_dns_guo
 * Readings (also in the numpy definition): the printed m_eq is for deviation
 * populations, so the rest-state moments rho0 (1, -11, 3, 0, ...) are added
 * for full populations; s_1 = s_e and s_9 = 1/tau0 enter eq. yu_strain
 * (tau_mode 0), or, self-consistently, the s_1 term is dropped and s_9 = 1/tau_e
 * (tau_mode 1, solved in closed form); the constant C enters nu_t linearly
 * unless smag_form = 1 (C^2).
 *
 * Data: full populations f[a][z][y][x], x fastest, a in the order of
 * App. B Fig. d3q19_table (0-based, rest last).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* App. B Fig. d3q19_table */
static const int CV[Q][3] = {
    {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {0, 1, 1},  {0, -1, -1},
    {0, 1, -1}, {0, -1, 1},  {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 0, 0}};
static const double WT[Q] = {
    1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 3};

/* App. B eq. moment-matrix, as printed */
static const double MM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, -30},
    {-4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 12},
    {1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0},
    {-4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 0},
    {0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 0},
    {0, 0, -4, 4, 0, 0, 1, -1, -1, 1, 1, -1, 1, -1, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0},
    {0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0},
    {2, 2, -1, -1, -1, -1, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1, 0},
    {-4, -4, 2, 2, 2, 2, 1, 1, 1, 1, -2, -2, -2, -2, 1, 1, 1, 1, 0},
    {0, 0, 1, 1, -1, -1, 1, 1, 1, 1, 0, 0, 0, 0, -1, -1, -1, -1, 0},
    {0, 0, -2, -2, 2, 2, 1, 1, 1, 1, 0, 0, 0, 0, -1, -1, -1, -1, 0},
    {0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0},
    {0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, -1, 1, -1, 1, 0},
    {0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 1, -1, -1, 1, 0}};

/* Parameters of one lattice (mirrored by a ctypes.Structure). */
typedef struct {
    int32_t nx, ny, nz, smag_form;
    double tau0, C, rho0;
    double s_e, s_eps, s_q, s_pi, s_m; /* eq. relaxation-matrix fixed rates */
    int32_t n_modes;
    int32_t tau_mode;          /* 0: s_9 = 1/tau0 in eq. yu_strain; 1: self-consistent */
    const int32_t* mode_k;     /* [n_modes][3] */
    const double* mode_amp;    /* [n_modes][3] */
    const double* mode_phase;  /* [n_modes]    */
} orc_params;

/* M^-1 = M^T diag(1/n_r), n_r = sum_a M_ra^2 (the rows of M are orthogonal). */
static double MINV[Q][Q];
static int minv_ready = 0;

static void build_minv(void) {
    if (minv_ready) return;
    for (int r = 0; r < Q; ++r) {
        double n = 0.0;
        for (int a = 0; a < Q; ++a) n += MM[r][a] * MM[r][a];
        for (int a = 0; a < Q; ++a) MINV[a][r] = MM[r][a] / n;
    }
    minv_ready = 1;
}

void orc_minv(double* out) {
    build_minv();
    memcpy(out, MINV, sizeof(MINV));
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Body force, the general form of Sec. 2.2 eq. forcing_pattern:
 * F = sum_m amp_m sin(2 pi (kx x/nx + ky y/ny + kz z/nz) + phase_m). */
void orc_force_at(const orc_params* p, int x, int y, int z, double F[3]) {
    F[0] = F[1] = F[2] = 0.0;
    for (int m = 0; m < p->n_modes; ++m) {
        const int32_t* k = p->mode_k + 3 * m;
        double arg = 2.0 * M_PI * ((double)k[0] * x / p->nx + (double)k[1] * y / p->ny +
                                   (double)k[2] * z / p->nz) +
                     p->mode_phase[m];
        double s = sin(arg);
        for (int a = 0; a < 3; ++a) F[a] += p->mode_amp[3 * m + a] * s;
    }
}

/* |S| of eq. strain_norm from the strain rate of eq. yu_strain (delta_t = 1)
 * with relaxation rates s1 (row 1) and s9 (rows 9, 11, 13-15). */
static double strain_norm_of(const double mneq[Q], double s1, double s9, double rho0) {
    const double Sxx = -(s1 * mneq[1] + 19.0 * s9 * mneq[9]) / (38.0 * rho0);
    const double Syy = -(2.0 * s1 * mneq[1] - 19.0 * s9 * (mneq[9] - 3.0 * mneq[11])) / (76.0 * rho0);
    const double Szz = -(2.0 * s1 * mneq[1] - 19.0 * s9 * (mneq[9] + 3.0 * mneq[11])) / (76.0 * rho0);
    const double Sxy = -3.0 * s9 / (2.0 * rho0) * mneq[13];
    const double Sxz = -3.0 * s9 / (2.0 * rho0) * mneq[15];
    const double Syz = -3.0 * s9 / (2.0 * rho0) * mneq[14];
    return sqrt(2.0 * (Sxx * Sxx + Syy * Syy + Szz * Szz +
                       2.0 * Sxy * Sxy + 2.0 * Sxz * Sxz + 2.0 * Syz * Syz));
}

/* One cell's collision (eq. mrt_les_guo).  Outputs the post-collision
 * populations and, optionally, rho, u (eq. guo_velocity) and tau_e. */
void orc_collide_cell(const orc_params* p, const double f[Q], const double F[3],
                      double fstar[Q], double* rho_out, double u_out[3], double* tau_out) {
    build_minv();
    const double rho0 = p->rho0;
    /* macroscopic quantities, eq. guo_velocity / eq. macroscopic_eq */
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        for (int d = 0; d < 3; ++d) j[d] += f[a] * CV[a][d];
    }
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / rho;
    const double ux = u[0], uy = u[1], uz = u[2];
    const double Fx = F[0], Fy = F[1], Fz = F[2];
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double drho = rho - rho0;

    /* moments m = M f */
    double m[Q];
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int a = 0; a < Q; ++a) s += MM[r][a] * f[a];
        m[r] = s;
    }

    /* equilibrium moments (printed deviation form) + rest-state offset */
    double meq[Q] = {drho,
                     -11.0 * drho + 19.0 * rho * u2,
                     -475.0 / 63.0 * rho * u2,
                     rho * ux, -2.0 * rho * ux / 3.0,
                     rho * uy, -2.0 * rho * uy / 3.0,
                     rho * uz, -2.0 * rho * uz / 3.0,
                     rho * (2.0 * ux * ux - uy * uy - uz * uz),
                     0.0,
                     rho * (uy * uy - uz * uz),
                     0.0,
                     rho * ux * uy, rho * uy * uz, rho * ux * uz,
                     0.0, 0.0, 0.0};
    meq[0] += rho0;
    meq[1] += -11.0 * rho0;
    meq[2] += 3.0 * rho0;

    /* force moments F_m */
    const double uF = ux * Fx + uy * Fy + uz * Fz;
    const double Fm[Q] = {0.0,
                          38.0 * uF, -11.0 * uF,
                          Fx, -2.0 * Fx / 3.0, Fy, -2.0 * Fy / 3.0, Fz, -2.0 * Fz / 3.0,
                          2.0 * (2.0 * ux * Fx - uy * Fy - uz * Fz),
                          -(2.0 * ux * Fx - uy * Fy - uz * Fz),
                          2.0 * (uy * Fy - uz * Fz),
                          -(uy * Fy - uz * Fz),
                          ux * Fy + uy * Fx, uy * Fz + uz * Fy, ux * Fz + uz * Fx,
                          0.0, 0.0, 0.0};

    double mneq[Q];
    for (int r = 0; r < Q; ++r) mneq[r] = m[r] - meq[r];

    /* eq. bare_viscosity, eq. eddy_visc, eq. les_viscosity (Delta = 1) */
    const double nu0 = (p->tau0 - 0.5) / 3.0;
    const double Cm = (p->smag_form == 1) ? p->C * p->C : p->C;
    double tau_e;
    if (p->tau_mode == 1) {
        /* S(s_1 = 0, s_9) = s_9 S(0, 1) and s_9 = 1/tau_e, so
         * tau_e = tau0 + 3 Cm |S(0, 1)| / tau_e: the positive root of the quadratic */
        const double S1 = strain_norm_of(mneq, 0.0, 1.0, rho0);
        tau_e = 0.5 * (p->tau0 + sqrt(p->tau0 * p->tau0 + 12.0 * Cm * S1));
    } else {
        const double Snorm = strain_norm_of(mneq, p->s_e, 1.0 / p->tau0, rho0);
        tau_e = 0.5 + 3.0 * (nu0 + Cm * Snorm);
    }
    const double s_nu = 1.0 / tau_e;

    /* eq. relaxation-matrix */
    const double S[Q] = {1.0, p->s_e, p->s_eps, 1.0, p->s_q, 1.0, p->s_q, 1.0, p->s_q,
                         s_nu, p->s_pi, s_nu, p->s_pi, s_nu, s_nu, s_nu,
                         p->s_m, p->s_m, p->s_m};

    double mstar[Q];
    for (int r = 0; r < Q; ++r) mstar[r] = m[r] - S[r] * mneq[r] + (1.0 - 0.5 * S[r]) * Fm[r];

    for (int a = 0; a < Q; ++a) {
        double s = 0.0;
        for (int r = 0; r < Q; ++r) s += MINV[a][r] * mstar[r];
        fstar[a] = s;
    }
    if (rho_out) *rho_out = rho;
    if (u_out) { u_out[0] = ux; u_out[1] = uy; u_out[2] = uz; }
    if (tau_out) *tau_out = tau_e;
}

static inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

/* The body force is static (Sec. 2.2), so it is evaluated once per call into
 * F[3][cells] and reused by every step of the call. */
static void force_field(const orc_params* p, double* F) {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t nc = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double Fc[3];
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                orc_force_at(p, x, y, z, Fc);
                F[c] = Fc[0]; F[nc + c] = Fc[1]; F[2 * nc + c] = Fc[2];
            }
        }
    }
}

/* One collide-and-stream step from f into g (push: g[a](x + c_a) = f*[a](x)). */
static void step_once(const orc_params* p, const double* F, const double* f, double* g) {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t nc = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double fc[Q], fs[Q], Fc[3];
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                for (int a = 0; a < Q; ++a) fc[a] = f[a * nc + c];
                Fc[0] = F[c]; Fc[1] = F[nc + c]; Fc[2] = F[2 * nc + c];
                orc_collide_cell(p, fc, Fc, fs, NULL, NULL, NULL);
                for (int a = 0; a < Q; ++a) {
                    const int xd = wrap(x + CV[a][0], nx);
                    const int yd = wrap(y + CV[a][1], ny);
                    const int zd = wrap(z + CV[a][2], nz);
                    g[a * nc + (size_t)xd + (size_t)nx * ((size_t)yd + (size_t)ny * zd)] = fs[a];
                }
            }
        }
    }
}

/* Advance f by nsteps; work has the same size as f (19 * nx*ny*nz doubles). */
int orc_step(const orc_params* p, double* f, double* work, int64_t nsteps) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || nsteps < 0) return -1;
    const size_t nc = (size_t)p->nx * p->ny * p->nz;
    const size_t n = (size_t)Q * nc;
    double* F = (double*)malloc(3 * nc * sizeof(double));
    if (!F) return -2;
    force_field(p, F);
    double* a = f;
    double* b = work;
    for (int64_t s = 0; s < nsteps; ++s) {
        step_once(p, F, a, b);
        double* t = a; a = b; b = t;
    }
    if (a != f) memcpy(f, a, n * sizeof(double));
    free(F);
    return 0;
}

/* Per-cell diagnostics of the state f (pre-collision): rho, u[3][cells], tau_e. */
void orc_fields(const orc_params* p, const double* f, double* rho, double* u, double* tau_e) {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t nc = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double fc[Q], fs[Q], F[3], uu[3], r, t;
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                for (int a = 0; a < Q; ++a) fc[a] = f[a * nc + c];
                orc_force_at(p, x, y, z, F);
                orc_collide_cell(p, fc, F, fs, &r, uu, &t);
                if (rho) rho[c] = r;
                if (u) { u[c] = uu[0]; u[nc + c] = uu[1]; u[2 * nc + c] = uu[2]; }
                if (tau_e) tau_e[c] = t;
            }
        }
    }
}

/* SplitMix64 (Steele, Lea & Flood 2014): the output for state v. */
uint64_t orc_splitmix64(uint64_t v) {
    uint64_t z = v + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* f(x, 0) = f_eq(rho0, u0(x)), App. A eq. feq.  kind: 0 noise, 1 TGV3D,
 * 2 TGV2D, 3 shear u_x = A sin(2 pi y/ny), 4 rest. */
int orc_init(const orc_params* p, int kind, double amp, uint64_t seed, double* f) {
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const size_t nc = (size_t)nx * ny * nz;
    if (kind < 0 || kind > 4) return -1;
    const uint64_t key = orc_splitmix64(seed);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                const size_t c = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                const double X = 2.0 * M_PI * x / nx, Y = 2.0 * M_PI * y / ny, Z = 2.0 * M_PI * z / nz;
                double u[3] = {0.0, 0.0, 0.0};
                if (kind == 1) {
                    u[0] = amp * sin(X) * cos(Y) * cos(Z);
                    u[1] = -amp * cos(X) * sin(Y) * cos(Z);
                } else if (kind == 2) {
                    u[0] = amp * sin(X) * cos(Y);
                    u[1] = -amp * cos(X) * sin(Y);
                } else if (kind == 3) {
                    u[0] = amp * sin(Y);
                } else if (kind == 0) {
                    for (int a = 0; a < 3; ++a) {
                        uint64_t h = orc_splitmix64(key ^ (3ULL * (uint64_t)c + (uint64_t)a));
                        double U = (double)(h >> 11) * 0x1.0p-53;
                        u[a] = amp * (2.0 * U - 1.0);
                    }
                }
                const double rho = p->rho0;
                const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                for (int a = 0; a < Q; ++a) {
                    const double cu = CV[a][0] * u[0] + CV[a][1] * u[1] + CV[a][2] * u[2];
                    f[a * nc + c] = WT[a] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
                }
            }
        }
    }
    return 0;
}

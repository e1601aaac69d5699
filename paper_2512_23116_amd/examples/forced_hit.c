/* forced_hit.c — the C-ABI of liblbm.so used from plain C (no Python, no torch).
 *
 * Runs the paper's LES setup on an N^3 periodic lattice (Sec. 3.1 and Sec. 4):
 * tau0 = 1/2 + 3 U0 N / Re with U0 = 0.043, the three-mode forcing of
 * eq. forcing_pattern with F0 = C_f U0^2 / N (C_f = 0.2), a Taylor-Green start
 * of amplitude U0, and prints the domain statistics of theta = tau_e - 1/2 and
 * K_t (Sec. 5.1) every `every` steps, then the shell spectrum E(1..4).
 *
 *   forced_hit [N=32] [steps=200] [every=100] [fp64|fp32|fp16|bf16] [aa|ab] [C=0.13] [Re=2e4]
 *
 * Output: one line per snapshot, "step <n> energy <E> theta_mean <..> theta_var <..>
 * kt_mean <..> kt_var <..> kt_flat <..> mass <..>" with %.17g values; exit status
 * 1 with the library's message on any error. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

static int check(lbm_status st, lbm_handle* h, const char* what) {
    if (st == LBM_OK) return 0;
    fprintf(stderr, "%s: %s (%s)\n", what, lbm_status_string(st), lbm_last_error(h));
    return 1;
}

int main(int argc, char** argv) {
    const int N = argc > 1 ? atoi(argv[1]) : 32;
    const long steps = argc > 2 ? atol(argv[2]) : 200;
    const long every = argc > 3 ? atol(argv[3]) : 100;
    const char* prec = argc > 4 ? argv[4] : "fp32";
    const char* scheme = argc > 5 ? argv[5] : "aa";
    const double C = argc > 6 ? atof(argv[6]) : 0.13;
    const double Re = argc > 7 ? atof(argv[7]) : 2.0e4;
    const double U0 = 0.043, F0 = 0.2 * U0 * U0 / N;
    if (N < 1 || steps < 0 || every < 1) {
        fprintf(stderr, "bad arguments\n");
        return 1;
    }

    lbm_config cfg;
    lbm_config_default(&cfg);
    cfg.nx = cfg.ny = cfg.nz = N;
    cfg.precision = !strcmp(prec, "fp64") ? LBM_FP64 : !strcmp(prec, "fp16") ? LBM_FP16_DEV
                  : !strcmp(prec, "bf16") ? LBM_BF16_DEV : LBM_FP32;
    cfg.streaming = !strcmp(scheme, "ab") ? LBM_STREAM_AB : LBM_STREAM_AA;
    cfg.smag_form = 1;
    cfg.tau0 = 0.5 + 3.0 * U0 * N / Re;
    cfg.smag_C = C;
    /* F_x = F0 sin(2 pi y / N), F_y = F0 sin(2 pi z / N), F_z = F0 sin(2 pi x / N) */
    lbm_force_mode modes[3];
    memset(modes, 0, sizeof modes);
    modes[0].k[1] = 1; modes[0].amp[0] = F0;
    modes[1].k[2] = 1; modes[1].amp[1] = F0;
    modes[2].k[0] = 1; modes[2].amp[2] = F0;
    cfg.n_force_modes = 3;
    cfg.force_modes = modes;

    lbm_handle* h = NULL;
    if (check(lbm_create(&cfg, &h), NULL, "lbm_create")) return 1;
    int rc = check(lbm_init_seeded(h, LBM_INIT_TGV3D, U0, 0), h, "lbm_init_seeded");
    for (long done = 0; !rc && done <= steps; done += every) {
        if (done > 0) rc = check(lbm_step(h, every), h, "lbm_step");
        lbm_stats s;
        if (!rc) rc = check(lbm_kt_stats(h, &s), h, "lbm_kt_stats");
        if (!rc)
            printf("step %lld energy %.17g theta_mean %.17g theta_var %.17g kt_mean %.17g "
                   "kt_var %.17g kt_flat %.17g mass %.17g\n", (long long)s.steps, s.energy,
                   s.theta_mean, s.theta_var, s.kt_mean, s.kt_var, s.kt_flat, s.mass);
    }
    double E[5];
    if (!rc) rc = check(lbm_spectrum(h, 4, E), h, "lbm_spectrum");
    if (!rc) printf("spectrum %.17g %.17g %.17g %.17g\n", E[1], E[2], E[3], E[4]);
    lbm_destroy(h);
    return rc;
}

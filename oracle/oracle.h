/*
 * FP64 CPU oracle of the RRRL iteration (test infrastructure only; see
 * oracle.c).  Images are row-major double arrays of H*W values, PSFs are
 * row-major double arrays of Py*Px taps with odd Py, Px.
 */
#ifndef DEBLUR_ORACLE_H
#define DEBLUR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_REPLICATE = 0, ORC_BC_PERIODIC = 1 };

typedef struct {
    double alpha;     /* regulariser weight (eq. (9)) */
    double eps_data;  /* epsilon of the data penaliser Phi */
    double eps_tv;    /* epsilon of the regulariser Psi */
    double s_min;     /* lower guard on the blurred iterate u*h */
    int robust;       /* 1: W = Phi'(r_f(u*h)); 0: W = 1 (plain RL data term) */
    int bc;           /* ORC_BC_* for the convolutions A and B */
    int psi;          /* regulariser: 0 regularised TV, 1 Perona-Malik (non-convex), lambda = eps_tv */
    int rf_lut;       /* 1: r_f through the lookup of Sec. 4.1 (orc_rf_lut); forward only */
} orc_params;

void orc_blur(const double* v, int H, int W, const double* h, int Py, int Px,
              int bc, double* out, int nthreads);
void orc_corr(const double* v, int H, int W, const double* h, int Py, int Px,
              int bc, double* out, int nthreads);
double orc_rf(double f, double s);
double orc_rf_lut(double f, double s);
void orc_tv(const double* u, int H, int W, double eps_t, int psi, double* D, int nthreads);
void orc_rrrl_step(const double* f, const double* u, double* u_next, int H, int W,
                   const double* h, int Py, int Px, const orc_params* p,
                   double* parts, int nthreads);
void orc_rrrl(const double* f, const double* u0, double* uK, int H, int W,
              const double* h, int Py, int Px, const orc_params* p, int iters,
              double* ckpt, int nthreads);

void orc_rrrl_step_adjoint(const double* f, const double* u, int H, int W, const double* h, int Py, int Px,
                           const orc_params* p, const double* lam, double* du, double* df, double* dh,
                           double* dalpha, int nthreads);

#ifdef __cplusplus
}
#endif
#endif

/* FP64 CPU oracle of the SPH hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and
 * its Python binding) includes, links or calls this code; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do. It shares no code
 * with the HIP path.
 *
 * What it computes (paper Sec. 2.1):
 *   * the density sum rho_i = sum_j m_j W(r_ij, h_i)            (Eq. density)
 *   * the discrete momentum equation with pressure gradient and
 *     artificial viscosity, and the matching internal-energy rate
 *                                                   (Eq. momentum, Eq. energy)
 *   * the linear kick/drift update                        (Alg. 1, CallLinear)
 *   * the AoS->SoA quantisers of Table 2 for the 32- and 16-bit rows and for
 *     bfloat16                                         (Sec. 3.2, Table 2)
 * The cubic-spline M4 kernel is the kernel family the paper names in Sec. 2.1.
 * Readings where the paper is silent are listed in the design notes and in
 * the comments of oracle.c.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double gamma_k;   /* support radius over smoothing length, H = gamma_k h  */
  double gamma;     /* adiabatic index of the ideal gas                     */
  double alpha;     /* artificial-viscosity strength                        */
  double beta;      /* signal-velocity coefficient of the viscosity         */
  int32_t gradh;    /* 1: grad-h correction factor f_i; 0: f_i = 1          */
  int32_t kernel;   /* ORC_KERNEL_M4 or ORC_KERNEL_WENDLAND_C2              */
} orc_params;

#define ORC_KERNEL_M4 0
#define ORC_KERNEL_WENDLAND_C2 1

/* dtype codes shared with the quantiser entry points */
enum { ORC_F32 = 0, ORC_F16 = 1, ORC_BF16 = 2, ORC_F64 = 3 };
/* truncate_mantissa storage of total size T bits (Sec. 3.2, Table 2):
 * dtype ORC_TRUNC + T, 9 <= T <= 64 */
enum { ORC_TRUNC = 0x100 };

/* kernel */
double orc_w_hat(double u);
double orc_dw_hat(double u);
double orc_W(double r, double h, double gamma_k);
double orc_dWdh(double r, double h, double gamma_k);
double orc_kernel_w(int kernel, double u);
double orc_kernel_dw(int kernel, double u);
double orc_W_k(int kernel, double r, double h, double gamma_k);
double orc_dWdh_k(int kernel, double r, double h, double gamma_k);

/* binning: wrap, integer cell, stable order by (cell, input index) */
int orc_bin(int n, const double *x, int n_c, int32_t *cell, int32_t *cell_start,
            int32_t *perm, double *off);

/* binning with sub-cell order: key = cell * R^3 + Morton(sub-cell), R = 2^sub_bits;
 * perm stable by (key, input index); sub_start[n_c^3 R^3 + 1] */
int orc_bin_sub(int n, const double *x, int n_c, int sub_bits, int32_t *key,
                int32_t *sub_start, int32_t *perm);

/* density; mode 0 = brute force over all pairs, 1 = own cell list.
 * sel (nsel entries) selects which i to evaluate; sel == NULL means all. */
int orc_density(int n, const double *x, const double *m, const double *h,
                const double *u, const orc_params *p, int mode, int n_c,
                const int32_t *sel, int nsel, const uint8_t *jmask, double *rho,
                double *wcount, double *rho_dh, double *f, double *P, double *c,
                int32_t *nngb);

int orc_force(int n, const double *x, const double *v, const double *m,
              const double *h, const double *rho, const double *f,
              const double *P, const double *c, const orc_params *p, int mode,
              int n_c, const int32_t *sel, int nsel, const uint8_t *jmask, double *a,
              double *du, double *vsig, int32_t *nforce);

void orc_kick_drift(int n, double *x, double *v, double *u, const double *a,
                    const double *du, double dt_kick, double dt_drift);

/* out[0..2] = sum m a; out[3] = sum m (v.a + du); out[4] = sum m |a|;
 * out[5] = sum m (|v.a| + |du|) */
void orc_reduce(int n, const double *m, const double *v, const double *a,
                const double *du, double *out);

/* smoothing lengths solving h = eta (m / rho(h))^(1/3) per particle */
int orc_smoothing_length(int n, const double *x, const double *m, const double *h0,
                         double eta, const orc_params *p, int mode, int n_c, double h_max,
                         double tol, int max_iter, const int32_t *sel, int nsel,
                         double *h_out, int32_t *iters);

/* per selected i, pairs whose FP64 separation lies within
 * eps_rel H + eps_abs of a support radius: near_d over the density list
 * (H_i), near_f over the force list (H_i or H_j, j != i) */
int orc_near_support(int n, const double *x, const double *h, double gamma_k, int mode,
                     int n_c, const int32_t *sel, int nsel, double eps_rel, double eps_abs,
                     int32_t *near_d, int32_t *near_f);

/* quantisers (RNE), FP32 -> {FP16, BF16} bits and back */
uint16_t orc_f32_to_f16(float v);
float orc_f16_to_f32(uint16_t b);
uint16_t orc_f32_to_bf16(float v);
float orc_bf16_to_f32(uint16_t b);
void orc_quant_array(int64_t n, const float *in, uint16_t *out, int dtype);
void orc_dequant_array(int64_t n, const uint16_t *in, float *out, int dtype);

/* FP64 value -> stored value -> FP64 (the value a kernel reads back) */
double orc_roundtrip(double v, int dtype, int scale);

/* position offsets from their anchor (0: cell corner; 1 + b: centre of the
 * sub-cell of side 1/(n_c 2^b)) and the anchor sub-cell code per particle */
int orc_pos_offsets(int n, const double *x, int n_c, int anchor, double *off, uint8_t *code);

/* Dequantised copy of a particle set as stored in an SoA view:
 * positions become anchor + stored offset, other fields round-trip. */
int orc_dequantise_set(int n, const double *x, const double *v, const double *m,
                       const double *h, const double *u, int n_c, int pos_dt,
                       int vel_dt, int mhu_dt, const int32_t *scales, int pos_anchor,
                       double *xq, double *vq, double *mq, double *hq, double *uq);

/* threads the OpenMP regions use, and setting them */
int orc_num_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif

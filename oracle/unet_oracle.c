/*
 * Plain FP64 CPU oracle of the U-Net layers of the learned initial guess.
 * TEST INFRASTRUCTURE ONLY (see qumond_oracle.c): the judge of the HIP
 * network kernels, sharing no code with them.
 *
 * Grids are vertex-centred n^3, channel-last: element (v, c) at v * C + c,
 * v = i + n (j + n k).  A 3x3x3 convolution with stride s and zero padding maps
 * an n_in^3 grid to n_out = (n_in - 1)/s + 1 points per side:
 *   y[o, co] = b[co] + sum_{d in {-1,0,1}^3} sum_ci x[s o + d, ci] w[co, d, ci]
 * with the tap index t = (dx+1) + 3 (dy+1) + 9 (dz+1) and w stored [co][t][ci].
 * The input and weight gradients are the adjoints of that map, written
 * directly from the definition (scatter over every output voxel and tap).
 */
#include <math.h>
#include <stddef.h>

static int inside(int i, int j, int k, int n) { return i >= 0 && j >= 0 && k >= 0 && i < n && j < n && k < n; }

void orc_conv3d_fwd(int nin, int cin, const double *x, int cout, const double *w, const double *b, int stride,
                    int relu, double *y)
{
    const int nout = (nin - 1) / stride + 1;
    for (int ko = 0; ko < nout; ko++)
        for (int jo = 0; jo < nout; jo++)
            for (int io = 0; io < nout; io++) {
                const size_t o = (size_t)io + (size_t)nout * (jo + (size_t)nout * ko);
                for (int co = 0; co < cout; co++) {
                    double s = b ? b[co] : 0.0;
                    for (int t = 0; t < 27; t++) {
                        const int i = stride * io + t % 3 - 1, j = stride * jo + (t / 3) % 3 - 1,
                                  k = stride * ko + t / 9 - 1;
                        if (!inside(i, j, k, nin)) continue;
                        const size_t v = (size_t)i + (size_t)nin * (j + (size_t)nin * k);
                        for (int ci = 0; ci < cin; ci++) s += x[v * cin + ci] * w[((size_t)co * 27 + t) * cin + ci];
                    }
                    if (relu && s < 0.0) s = 0.0;
                    y[o * cout + co] = s;
                }
            }
}

void orc_conv3d_dgrad(int nin, int cin, int cout, const double *w, int stride, const double *dy, double *dx)
{
    const int nout = (nin - 1) / stride + 1;
    const size_t N = (size_t)nin * nin * nin;
    for (size_t q = 0; q < N * cin; q++) dx[q] = 0.0;
    for (int ko = 0; ko < nout; ko++)
        for (int jo = 0; jo < nout; jo++)
            for (int io = 0; io < nout; io++) {
                const size_t o = (size_t)io + (size_t)nout * (jo + (size_t)nout * ko);
                for (int t = 0; t < 27; t++) {
                    const int i = stride * io + t % 3 - 1, j = stride * jo + (t / 3) % 3 - 1, k = stride * ko + t / 9 - 1;
                    if (!inside(i, j, k, nin)) continue;
                    const size_t v = (size_t)i + (size_t)nin * (j + (size_t)nin * k);
                    for (int co = 0; co < cout; co++) {
                        const double g = dy[o * cout + co];
                        for (int ci = 0; ci < cin; ci++) dx[v * cin + ci] += g * w[((size_t)co * 27 + t) * cin + ci];
                    }
                }
            }
}

void orc_conv3d_wgrad(int nin, int cin, const double *x, int cout, const double *dy, int stride, double *dw)
{
    const int nout = (nin - 1) / stride + 1;
    for (size_t q = 0; q < (size_t)cout * 27 * cin; q++) dw[q] = 0.0;
    for (int ko = 0; ko < nout; ko++)
        for (int jo = 0; jo < nout; jo++)
            for (int io = 0; io < nout; io++) {
                const size_t o = (size_t)io + (size_t)nout * (jo + (size_t)nout * ko);
                for (int t = 0; t < 27; t++) {
                    const int i = stride * io + t % 3 - 1, j = stride * jo + (t / 3) % 3 - 1, k = stride * ko + t / 9 - 1;
                    if (!inside(i, j, k, nin)) continue;
                    const size_t v = (size_t)i + (size_t)nin * (j + (size_t)nin * k);
                    for (int co = 0; co < cout; co++) {
                        const double g = dy[o * cout + co];
                        for (int ci = 0; ci < cin; ci++) dw[((size_t)co * 27 + t) * cin + ci] += g * x[v * cin + ci];
                    }
                }
            }
}

/* Trilinear 2x up-sampling (vertex-centred, n_fine = 2 n_coarse - 1) and its adjoint. */
static double wt1(int f, int c) { return f == 2 * c ? 1.0 : ((f == 2 * c - 1 || f == 2 * c + 1) ? 0.5 : 0.0); }

void orc_upsample(int nc, int ch, const double *xc, double *xf)
{
    const int nf = 2 * nc - 1;
    for (int k = 0; k < nf; k++)
        for (int j = 0; j < nf; j++)
            for (int i = 0; i < nf; i++) {
                const size_t v = (size_t)i + (size_t)nf * (j + (size_t)nf * k);
                for (int c = 0; c < ch; c++) xf[v * ch + c] = 0.0;
                for (int K = k / 2; K <= (k + 1) / 2; K++)
                    for (int J = j / 2; J <= (j + 1) / 2; J++)
                        for (int I = i / 2; I <= (i + 1) / 2; I++) {
                            const double w = wt1(i, I) * wt1(j, J) * wt1(k, K);
                            const size_t u = (size_t)I + (size_t)nc * (J + (size_t)nc * K);
                            for (int c = 0; c < ch; c++) xf[v * ch + c] += w * xc[u * ch + c];
                        }
            }
}

void orc_upsample_adj(int nc, int ch, const double *gf, double *gc)
{
    const int nf = 2 * nc - 1;
    for (size_t q = 0; q < (size_t)nc * nc * nc * ch; q++) gc[q] = 0.0;
    for (int k = 0; k < nf; k++)
        for (int j = 0; j < nf; j++)
            for (int i = 0; i < nf; i++) {
                const size_t v = (size_t)i + (size_t)nf * (j + (size_t)nf * k);
                for (int K = k / 2; K <= (k + 1) / 2; K++)
                    for (int J = j / 2; J <= (j + 1) / 2; J++)
                        for (int I = i / 2; I <= (i + 1) / 2; I++) {
                            const double w = wt1(i, I) * wt1(j, J) * wt1(k, K);
                            const size_t u = (size_t)I + (size_t)nc * (J + (size_t)nc * K);
                            for (int c = 0; c < ch; c++) gc[u * ch + c] += w * gf[v * ch + c];
                        }
            }
}

/*
 * One step of Adam (Kingma and Ba, "Adam: a method for stochastic
 * optimization", ICLR 2015, Algorithm 1) on `count` parameters, in FP64: with
 * the gradient g of step t (t >= 1, counted from 1),
 *   m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
 *   m_hat = m / (1 - b1^t),   v_hat = v / (1 - b2^t),
 *   w <- w - lr m_hat / (sqrt(v_hat) + eps).
 * m and v start at zero before step 1.
 */
void orc_adam_step(int count, double *w, double *m, double *v, const double *g, double lr, double b1, double b2,
                   double eps, int t)
{
    double c1 = 1.0, c2 = 1.0;
    for (int s = 0; s < t; s++) {   /* b1^t and b2^t by repeated products */
        c1 *= b1;
        c2 *= b2;
    }
    c1 = 1.0 - c1;
    c2 = 1.0 - c2;
    for (int i = 0; i < count; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        const double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/*
 * mlp_oracle.c -- plain FP64 reference of the warm-start network.
 *
 * TEST INFRASTRUCTURE ONLY (loaded by the tests; shares nothing with the GPU
 * library).  A fully connected network 5 -> H -> ... -> H -> 3 (`depth`
 * hidden layers, SiLU activation s(z) = z / (1 + exp(-z)), linear output),
 * the mean-squared-error loss over the batch and the three outputs, its
 * gradient by backpropagation, and one Adam update (Kingma & Ba 2015).
 *
 * Pins: the gradient against central differences of the loss, a network with
 * zero parameters predicts zero, the forward pass of a one-hidden-layer
 * network worked by hand, and the first Adam step in closed form
 * (-lr sign(g) up to eps).
 *
 * Parameter order: for each layer l = 0..depth, W_l as [n_out][n_in]
 * row-major, then b_l [n_out].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NIN 5
#define NOUT 3

static int layer_in(int l, int H) { return l == 0 ? NIN : H; }
static int layer_out(int l, int H, int depth) { return l == depth ? NOUT : H; }

long mlp_num_params(int H, int depth)
{
    long n = 0;
    for (int l = 0; l <= depth; ++l) n += (long)layer_out(l, H, depth) * layer_in(l, H) + layer_out(l, H, depth);
    return n;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }
static double dsilu(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

/* Forward pass of n samples: x [n][5] -> y [n][3]. */
void mlp_forward(const double *p, int H, int depth, const double *x, long n, double *y)
{
    double *a = (double *)malloc(sizeof(double) * (H > NIN ? H : NIN));
    double *z = (double *)malloc(sizeof(double) * H);
    for (long s = 0; s < n; ++s) {
        memcpy(a, x + s * NIN, sizeof(double) * NIN);
        const double *q = p;
        for (int l = 0; l <= depth; ++l) {
            int ni = layer_in(l, H), no = layer_out(l, H, depth);
            const double *W = q, *b = q + (long)no * ni;
            for (int j = 0; j < no; ++j) {
                double acc = b[j];
                for (int i = 0; i < ni; ++i) acc += W[(long)j * ni + i] * a[i];
                z[j] = acc;
            }
            q += (long)no * ni + no;
            if (l == depth)
                for (int j = 0; j < no; ++j) y[s * NOUT + j] = z[j];
            else
                for (int j = 0; j < no; ++j) a[j] = silu(z[j]);
        }
    }
    free(a); free(z);
}

/* Loss L = 1/(3n) sum (y - t)^2 and its gradient dL/dp (same order as p). */
double mlp_gradient(const double *p, int H, int depth, const double *x, const double *t, long n, double *grad)
{
    const long np = mlp_num_params(H, depth);
    memset(grad, 0, sizeof(double) * np);
    /* per-layer pre-activations and activations of one sample */
    double *A = (double *)malloc(sizeof(double) * (depth + 1) * (H > NIN ? H : NIN));
    double *Z = (double *)malloc(sizeof(double) * (depth + 1) * H);
    double *d = (double *)malloc(sizeof(double) * H);
    double *dn = (double *)malloc(sizeof(double) * H);
    long *off = (long *)malloc(sizeof(long) * (depth + 1));
    const int AW = H > NIN ? H : NIN;
    long o = 0;
    for (int l = 0; l <= depth; ++l) {
        off[l] = o;
        o += (long)layer_out(l, H, depth) * layer_in(l, H) + layer_out(l, H, depth);
    }
    double loss = 0.0;
    for (long s = 0; s < n; ++s) {
        memcpy(A, x + s * NIN, sizeof(double) * NIN);
        for (int l = 0; l <= depth; ++l) {
            int ni = layer_in(l, H), no = layer_out(l, H, depth);
            const double *W = p + off[l], *b = W + (long)no * ni;
            for (int j = 0; j < no; ++j) {
                double acc = b[j];
                for (int i = 0; i < ni; ++i) acc += W[(long)j * ni + i] * A[l * AW + i];
                Z[l * H + j] = acc;
                if (l < depth) A[(l + 1) * AW + j] = silu(acc);
            }
        }
        /* output layer is linear: dL/dz = 2 (y - t) / (3 n) */
        for (int j = 0; j < NOUT; ++j) {
            double e = Z[depth * H + j] - t[s * NOUT + j];
            loss += e * e;
            d[j] = 2.0 * e / (3.0 * (double)n);
        }
        for (int l = depth; l >= 0; --l) {
            int ni = layer_in(l, H), no = layer_out(l, H, depth);
            const double *W = p + off[l];
            double *gW = grad + off[l], *gb = gW + (long)no * ni;
            for (int j = 0; j < no; ++j) {
                gb[j] += d[j];
                for (int i = 0; i < ni; ++i) gW[(long)j * ni + i] += d[j] * A[l * AW + i];
            }
            if (l > 0) {
                for (int i = 0; i < ni; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < no; ++j) acc += W[(long)j * ni + i] * d[j];
                    dn[i] = acc * dsilu(Z[(l - 1) * H + i]);
                }
                memcpy(d, dn, sizeof(double) * ni);
            }
        }
    }
    free(A); free(Z); free(d); free(dn); free(off);
    return loss / (3.0 * (double)n);
}

/* One Adam step (step count t >= 1). */
void mlp_adam(double *p, const double *g, double *m, double *v, long np, double lr, double b1, double b2,
              double eps, long t)
{
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long k = 0; k < np; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        p[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}

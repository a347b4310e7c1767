/*
 * CPU oracle of the collision-surrogate MLP -- TEST INFRASTRUCTURE ONLY.
 *
 * The surrogate is not part of the paper: it is this build's learned
 * pre-filter for the static-scene overlap test of the kinematic step
 * (Section 3.2).  Network: input x (2112 values) -> 4 hidden layers of 256
 * units with ReLU -> one logit z; p = sigmoid(z).  On the device, weights and
 * activations are BF16 with FP32 accumulation; this oracle evaluates the same
 * network in FP64 on the same BF16 values, rounding activations (and the
 * back-propagated pre-activation gradients) to BF16 at the points where the
 * device does, or not at all ("exact" mode, used for finite differences).
 *
 * Layer l (1..5) maps dims[l-1] inputs to dims[l] outputs:
 *   pre_l = W_l h_{l-1} + b_l,  h_l = bf16(relu(pre_l)) for l <= 4,  z = pre_5.
 * W_l is stored [dims[l]][dims[l-1]] (one row per output unit).
 * Loss (per row i, weight w_i = pos_weight if y_i = 1 else 1):
 *   L = (1/B) sum_i w_i * (max(z,0) - z*y + log(1 + exp(-|z|)))   (logistic loss)
 * Backward: dz_i = w_i (sigmoid(z_i) - y_i) / B; for l = 5..1
 *   dW_l = sum_i dpre_l[i] h_{l-1}[i]^T, db_l = sum_i dpre_l[i],
 *   dpre_{l-1} = bf16((W_l^T dpre_l) * [h_{l-1} > 0]).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_EXPORT __attribute__((visibility("default")))

/* round to the nearest BF16 value (8 significant bits), ties to even */
O_EXPORT double o_bf16_round(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    double m = frexp(v, &e);            /* v = m * 2^e, 0.5 <= |m| < 1 */
    double s = ldexp(m, 8);             /* 8 significant bits */
    double r = nearbyint(s);            /* current rounding mode: to nearest, ties even */
    return ldexp(r, e - 8);
}

typedef struct {
    int32_t dims[6];                    /* input, 4 hidden, output (1) */
    const double *W[5];                 /* [dims[l+1]][dims[l]] */
    const double *b[5];                 /* [dims[l+1]] */
} o_mlp;

static double relu(double v) { return v > 0.0 ? v : 0.0; }

/* acts: optional [sum over l=1..4 of rows*dims[l]] storage of h_1..h_4 */
O_EXPORT void o_mlp_forward(const o_mlp *net, const double *x, int rows, int round_bf16,
                            double *logits, double *acts)
{
    const int D0 = net->dims[0];
    int maxd = 0;
    for (int l = 0; l < 6; ++l) if (net->dims[l] > maxd) maxd = net->dims[l];
    double *cur = malloc(sizeof(double) * (size_t)maxd);
    double *nxt = malloc(sizeof(double) * (size_t)maxd);
    size_t aoff = 0;
    for (int i = 0; i < rows; ++i) {
        memcpy(cur, x + (size_t)i * D0, sizeof(double) * (size_t)D0);
        for (int l = 0; l < 5; ++l) {
            const int din = net->dims[l], dout = net->dims[l + 1];
            for (int o = 0; o < dout; ++o) {
                double acc = net->b[l][o];
                const double *w = net->W[l] + (size_t)o * din;
                for (int k = 0; k < din; ++k) acc += w[k] * cur[k];
                if (l < 4) {
                    double h = relu(acc);
                    nxt[o] = round_bf16 ? o_bf16_round(h) : h;
                } else {
                    nxt[o] = acc;
                }
            }
            if (l < 4 && acts) {
                size_t base = 0;
                for (int q = 1; q <= l; ++q) base += (size_t)rows * net->dims[q];
                memcpy(acts + base + (size_t)i * dout, nxt, sizeof(double) * (size_t)dout);
            }
            double *t = cur; cur = nxt; nxt = t;
        }
        logits[i] = cur[0];
    }
    (void)aoff;
    free(cur);
    free(nxt);
}

static double logistic_loss(double z, double y)
{
    return (z > 0.0 ? z : 0.0) - z * y + log1p(exp(-fabs(z)));
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Gradients of the weighted logistic loss.  dW[l] has the shape of W[l],
   db[l] of b[l]; returns the loss. */
O_EXPORT double o_mlp_backward(const o_mlp *net, const double *x, const double *labels, int rows,
                               double pos_weight, int round_bf16, double **dW, double **db)
{
    size_t total = 0;
    for (int l = 1; l <= 4; ++l) total += (size_t)rows * net->dims[l];
    double *acts = malloc(sizeof(double) * (total ? total : 1));
    double *z = malloc(sizeof(double) * (size_t)rows);
    o_mlp_forward(net, x, rows, round_bf16, z, acts);
    const double *h[5];
    h[0] = x;
    size_t off = 0;
    for (int l = 1; l <= 4; ++l) {
        h[l] = acts + off;
        off += (size_t)rows * net->dims[l];
    }
    for (int l = 0; l < 5; ++l) {
        memset(dW[l], 0, sizeof(double) * (size_t)net->dims[l + 1] * net->dims[l]);
        memset(db[l], 0, sizeof(double) * (size_t)net->dims[l + 1]);
    }
    int maxd = 0;
    for (int l = 0; l < 6; ++l) if (net->dims[l] > maxd) maxd = net->dims[l];
    double *dpre = malloc(sizeof(double) * (size_t)maxd);
    double *dh = malloc(sizeof(double) * (size_t)maxd);
    double loss = 0.0;
    for (int i = 0; i < rows; ++i) {
        const double w = labels[i] > 0.5 ? pos_weight : 1.0;
        loss += w * logistic_loss(z[i], labels[i]);
        dpre[0] = w * (sigmoid(z[i]) - labels[i]) / rows;
        for (int l = 4; l >= 0; --l) {
            const int din = net->dims[l], dout = net->dims[l + 1];
            const double *hin = h[l] + (size_t)i * din;
            for (int o = 0; o < dout; ++o) {
                db[l][o] += dpre[o];
                double *g = dW[l] + (size_t)o * din;
                for (int k = 0; k < din; ++k) g[k] += dpre[o] * hin[k];
            }
            if (l == 0) break;
            for (int k = 0; k < din; ++k) {
                double acc = 0.0;
                for (int o = 0; o < dout; ++o) acc += net->W[l][(size_t)o * din + k] * dpre[o];
                double v = hin[k] > 0.0 ? acc : 0.0;
                dh[k] = round_bf16 ? o_bf16_round(v) : v;
            }
            memcpy(dpre, dh, sizeof(double) * (size_t)din);
        }
    }
    free(dpre);
    free(dh);
    free(acts);
    free(z);
    return loss / rows;
}

O_EXPORT double o_mlp_loss(const o_mlp *net, const double *x, const double *labels, int rows,
                           double pos_weight, int round_bf16)
{
    double *z = malloc(sizeof(double) * (size_t)rows);
    o_mlp_forward(net, x, rows, round_bf16, z, NULL);
    double loss = 0.0;
    for (int i = 0; i < rows; ++i)
        loss += (labels[i] > 0.5 ? pos_weight : 1.0) * logistic_loss(z[i], labels[i]);
    free(z);
    return loss / rows;
}

/* One Adam step (Kingma & Ba 2015) on FP64 copies, for comparison with the
   device update of the FP32 master weights. */
O_EXPORT void o_adam(double *w, double *m, double *v, const double *g, int64_t n, double lr,
                     double beta1, double beta2, double eps, int64_t t)
{
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        const double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

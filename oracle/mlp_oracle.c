/*
 * mlp_oracle.c -- CPU reference for the flow-map surrogate network.
 *
 * TEST INFRASTRUCTURE: loaded only by the test-suite; the GPU library never
 * links or calls it.
 *
 * The network (not part of the paper; a learned stand-in for the RK4 trace):
 *   input  x in R^4 (scaled position and time)
 *   z1 = W1 x + b1,  a1 = gelu(z1)          (4 -> 64)
 *   z2 = W2 a1 + b2, a2 = gelu(z2)          (64 -> 64)
 *   z3 = W3 a2 + b3, a3 = gelu(z3)          (64 -> 64)
 *   y  = W4 a3 + b4                         (64 -> 3)
 * gelu(u) = u/2 (1 + tanh(sqrt(2/pi) (u + 0.044715 u^3)))   (tanh form of
 * Hendrycks & Gimpel, 2016).  Loss: L = 1/(3B) sum_i |y_i - t_i|^2.
 * Parameters, flat, layer by layer: W1[64][4] b1[64] W2[64][64] b2[64]
 * W3[64][64] b3[64] W4[3][64] b4[3] (W[out][in]).
 *
 * bf16 mode reproduces where the GPU rounds to bfloat16 (round to nearest,
 * ties to even): W2, W3 and the matrix-core operands a1, a2 in the forward
 * pass; in the backward pass the matrix-core operands dz3, dz2 (and W2, W3,
 * a1, a2 again).  Everything else is float64 here.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define H 64
#define NP (4 * H + H + 2 * (H * H + H) + H * 3 + 3)

int64_t orc_mlp_nparams(void) { return NP; }

double orc_bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;  /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return f;
}

double orc_gelu(double u)
{
    const double c = sqrt(2.0 / M_PI);
    return 0.5 * u * (1.0 + tanh(c * (u + 0.044715 * u * u * u)));
}

static double gelu_d(double u)
{
    const double c = sqrt(2.0 / M_PI);
    double inner = c * (u + 0.044715 * u * u * u);
    double th = tanh(inner);
    double dinner = c * (1.0 + 3.0 * 0.044715 * u * u);
    return 0.5 * (1.0 + th) + 0.5 * u * (1.0 - th * th) * dinner;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
} net;

static net unpack(const double *p)
{
    net n;
    n.W1 = p;
    n.b1 = n.W1 + 4 * H;
    n.W2 = n.b1 + H;
    n.b2 = n.W2 + H * H;
    n.W3 = n.b2 + H;
    n.b3 = n.W3 + H * H;
    n.W4 = n.b3 + H;
    n.b4 = n.W4 + 3 * H;
    return n;
}

static double rb(double v, int bf) { return bf ? orc_bf16_round(v) : v; }

/* one sample: forward pass with the stored intermediates */
static void fwd1(const net *n, const double *x, int bf, double *z1, double *a1, double *z2, double *a2, double *z3,
                 double *a3, double *y)
{
    for (int o = 0; o < H; ++o) {
        double acc = n->b1[o];
        for (int i = 0; i < 4; ++i) acc += n->W1[o * 4 + i] * x[i];
        z1[o] = acc;
        a1[o] = orc_gelu(acc);
    }
    for (int o = 0; o < H; ++o) {
        double acc = 0;
        for (int i = 0; i < H; ++i) acc += rb(n->W2[o * H + i], bf) * rb(a1[i], bf);
        z2[o] = acc + n->b2[o];
        a2[o] = orc_gelu(z2[o]);
    }
    for (int o = 0; o < H; ++o) {
        double acc = 0;
        for (int i = 0; i < H; ++i) acc += rb(n->W3[o * H + i], bf) * rb(a2[i], bf);
        z3[o] = acc + n->b3[o];
        a3[o] = orc_gelu(z3[o]);
    }
    for (int o = 0; o < 3; ++o) {
        double acc = n->b4[o];
        for (int i = 0; i < H; ++i) acc += n->W4[o * H + i] * a3[i];
        y[o] = acc;
    }
}

/* y[n][3] = net(x[n][4]) */
void orc_mlp_forward(const double *params, int64_t nsamp, const double *x, double *y, int bf16)
{
    net n = unpack(params);
    double z1[H], a1[H], z2[H], a2[H], z3[H], a3[H];
    for (int64_t s = 0; s < nsamp; ++s) fwd1(&n, x + 4 * s, bf16, z1, a1, z2, a2, z3, a3, y + 3 * s);
}

/* loss and gradient (grad[NP], overwritten) over nsamp samples */
double orc_mlp_loss_grad(const double *params, int64_t nsamp, const double *x, const double *t, double *grad, int bf16)
{
    net n = unpack(params);
    net g;
    memset(grad, 0, sizeof(double) * NP);
    g = unpack(grad);
    double *gW1 = (double *)g.W1, *gb1 = (double *)g.b1, *gW2 = (double *)g.W2, *gb2 = (double *)g.b2;
    double *gW3 = (double *)g.W3, *gb3 = (double *)g.b3, *gW4 = (double *)g.W4, *gb4 = (double *)g.b4;
    double loss = 0;
    const double scale = 1.0 / (3.0 * (double)nsamp);
    for (int64_t s = 0; s < nsamp; ++s) {
        const double *xs = x + 4 * s, *ts = t + 3 * s;
        double z1[H], a1[H], z2[H], a2[H], z3[H], a3[H], y[3];
        fwd1(&n, xs, bf16, z1, a1, z2, a2, z3, a3, y);
        double dy[3];
        for (int o = 0; o < 3; ++o) {
            double e = y[o] - ts[o];
            loss += e * e * scale;
            dy[o] = 2.0 * e * scale;
        }
        /* layer 4 */
        double da3[H];
        for (int i = 0; i < H; ++i) da3[i] = 0;
        for (int o = 0; o < 3; ++o) {
            gb4[o] += dy[o];
            for (int i = 0; i < H; ++i) {
                gW4[o * H + i] += dy[o] * a3[i];
                da3[i] += dy[o] * n.W4[o * H + i];
            }
        }
        /* layer 3 */
        double dz3[H], da2[H];
        for (int o = 0; o < H; ++o) dz3[o] = da3[o] * gelu_d(z3[o]);
        for (int i = 0; i < H; ++i) da2[i] = 0;
        for (int o = 0; o < H; ++o) {
            double d = rb(dz3[o], bf16);
            gb3[o] += dz3[o];
            for (int i = 0; i < H; ++i) {
                gW3[o * H + i] += d * rb(a2[i], bf16);
                da2[i] += d * rb(n.W3[o * H + i], bf16);
            }
        }
        /* layer 2 */
        double dz2[H], da1[H];
        for (int o = 0; o < H; ++o) dz2[o] = da2[o] * gelu_d(z2[o]);
        for (int i = 0; i < H; ++i) da1[i] = 0;
        for (int o = 0; o < H; ++o) {
            double d = rb(dz2[o], bf16);
            gb2[o] += dz2[o];
            for (int i = 0; i < H; ++i) {
                gW2[o * H + i] += d * rb(a1[i], bf16);
                da1[i] += d * rb(n.W2[o * H + i], bf16);
            }
        }
        /* layer 1 */
        for (int o = 0; o < H; ++o) {
            double dz1 = da1[o] * gelu_d(z1[o]);
            gb1[o] += dz1;
            for (int i = 0; i < 4; ++i) gW1[o * 4 + i] += dz1 * xs[i];
        }
    }
    return loss;
}

/* Adam (Kingma & Ba 2015), step count t >= 1, bias-corrected */
void orc_adam_step(double *p, const double *g, double *m, double *v, int64_t n, double lr, double b1, double b2,
                   double eps, int64_t t)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

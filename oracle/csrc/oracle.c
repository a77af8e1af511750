/*
 * Oracle: plain, slow, single-threaded FP64 point operations of the loop-chain
 * workloads.  TEST INFRASTRUCTURE ONLY: nothing in the product library links,
 * includes or calls this file.
 *
 * Each function executes ONE parallel loop over its whole iteration range,
 * point by point, in plain nested loops (x fastest).  The order of the terms
 * in every point formula is fixed and written out with explicit fma() (C99,
 * correctly rounded) or plain + - * / so that the result of each point is
 * fully determined.  Compiled with -O2 -ffp-contract=off so that the compiler
 * adds no contractions of its own.
 *
 * Array view: element (x,y,z) (logical coordinates, halo points negative or
 * >= size) lives at p[origin + x*sx + y*sy + z*sz].
 *
 * Loop semantics follow the parallel-loop abstraction of the paper (Section 3:
 * a user kernel applied at every point of an iteration range, each argument a
 * dataset accessed through a stencil, read / written / incremented).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    double *p;
    int64_t origin;
    int64_t sx, sy, sz;
} ov;

#define AT(v, x, y, z) ((v).p[(v).origin + (int64_t)(x) * (v).sx + (int64_t)(y) * (v).sy + (int64_t)(z) * (v).sz])

/* Weighted sum of stencil reads:
 *   acc = 0; for each input a (listed order), for each stencil point q (listed
 *   order): acc = fma(w[a][q], in_a[x + off_q], acc);  out[x] = acc.
 * offs holds 3 ints per point (x,y,z offsets), inputs back to back. */
int orc_wsum(const int64_t lo[3], const int64_t hi[3], ov out, int nin, const ov *in,
             const int *npts, const int *offs, const double *w)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double acc = 0.0;
                int q = 0;
                for (int a = 0; a < nin; ++a)
                    for (int k = 0; k < npts[a]; ++k, ++q) {
                        const int *o = offs + 3 * q;
                        acc = fma(w[q], AT(in[a], x + o[0], y + o[1], z + o[2]), acc);
                    }
                AT(out, x, y, z) = acc;
            }
    return 0;
}

/* out = in */
int orc_copy(const int64_t lo[3], const int64_t hi[3], ov out, ov in)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x)
                AT(out, x, y, z) = AT(in, x, y, z);
    return 0;
}

/* y = fma(a, x, b*y) */
int orc_axpby(const int64_t lo[3], const int64_t hi[3], ov yv, ov xv, double a, double b)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x)
                AT(yv, x, y, z) = fma(a, AT(xv, x, y, z), b * AT(yv, x, y, z));
    return 0;
}

/* Reflective ghost fill along one axis.  Low side: ghost coordinate c = -1-i
 * takes the value at i = -1-c.  High side (size n along the axis): c = n+i
 * takes the value at n-1-i = 2n-1-c.  Only the iteration range is written. */
int orc_halo_reflect(const int64_t lo[3], const int64_t hi[3], ov v, int axis, int side, int64_t n)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                int64_t c[3] = {x, y, z};
                int64_t s[3] = {x, y, z};
                s[axis] = side == 0 ? -1 - c[axis] : 2 * n - 1 - c[axis];
                AT(v, x, y, z) = AT(v, s[0], s[1], s[2]);
            }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Heat-conduction operator (reflective boundaries), 2D or 3D.
 * K[d] is the face coefficient on the low face of the cell along axis d.
 *   diag = 1 + K0(+x) + K0(0) + K1(+y) + K1(0) [+ K2(+z) + K2(0)]   (left to right)
 *   Av = diag*v; then Av = fma(-K, v_nb, Av) for E, W, N, S [, T, B] in order. */
static double tea_apply(int nd, const ov *K, ov v, int64_t x, int64_t y, int64_t z)
{
    double ke = AT(K[0], x + 1, y, z), kw = AT(K[0], x, y, z);
    double kn = AT(K[1], x, y + 1, z), ks = AT(K[1], x, y, z);
    double diag = 1.0 + ke;
    diag = diag + kw;
    diag = diag + kn;
    diag = diag + ks;
    double kt = 0.0, kb = 0.0;
    if (nd == 3) {
        kt = AT(K[2], x, y, z + 1);
        kb = AT(K[2], x, y, z);
        diag = diag + kt;
        diag = diag + kb;
    }
    double av = diag * AT(v, x, y, z);
    av = fma(-ke, AT(v, x + 1, y, z), av);
    av = fma(-kw, AT(v, x - 1, y, z), av);
    av = fma(-kn, AT(v, x, y + 1, z), av);
    av = fma(-ks, AT(v, x, y - 1, z), av);
    if (nd == 3) {
        av = fma(-kt, AT(v, x, y, z + 1), av);
        av = fma(-kb, AT(v, x, y, z - 1), av);
    }
    return av;
}

/* u0 = e * rho; u = u0 */
int orc_tea_init(const int64_t lo[3], const int64_t hi[3], ov rho, ov e, ov u0, ov u)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double t = AT(e, x, y, z) * AT(rho, x, y, z);
                AT(u0, x, y, z) = t;
                AT(u, x, y, z) = t;
            }
    return 0;
}

/* Face coefficients: K_d(c) = (2*r) / (rho(c - e_d) + rho(c)), harmonic mean of
 * the conductivity 1/rho of the two cells sharing the low face along axis d. */
int orc_tea_k(int nd, const int64_t lo[3], const int64_t hi[3], ov rho, const ov *K, double r)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double c = AT(rho, x, y, z);
                AT(K[0], x, y, z) = (2.0 * r) / (AT(rho, x - 1, y, z) + c);
                AT(K[1], x, y, z) = (2.0 * r) / (AT(rho, x, y - 1, z) + c);
                if (nd == 3)
                    AT(K[2], x, y, z) = (2.0 * r) / (AT(rho, x, y, z - 1) + c);
            }
    return 0;
}

/* r = b - A x */
int orc_tea_resid(int nd, const int64_t lo[3], const int64_t hi[3], const ov *K, ov xv, ov b, ov r)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x)
                AT(r, x, y, z) = AT(b, x, y, z) - tea_apply(nd, K, xv, x, y, z);
    return 0;
}

/* w = A p; contribution p*w split exactly into (prod, err) per point, written
 * to c[2*i], c[2*i+1] in point order (the caller sums them exactly). */
int orc_tea_matvec_dot(int nd, const int64_t lo[3], const int64_t hi[3], const ov *K, ov p, ov w, double *c)
{
    int64_t i = 0;
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x, ++i) {
                double a = tea_apply(nd, K, p, x, y, z);
                AT(w, x, y, z) = a;
                double pv = AT(p, x, y, z);
                double pr = pv * a;
                c[2 * i] = pr;
                c[2 * i + 1] = fma(pv, a, -pr);
            }
    return 0;
}

/* rt = rt - A sd; z = z + sd */
int orc_tea_p1(int nd, const int64_t lo[3], const int64_t hi[3], const ov *K, ov sd, ov rt, ov zv)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double a = tea_apply(nd, K, sd, x, y, z);
                AT(rt, x, y, z) = AT(rt, x, y, z) - a;
                AT(zv, x, y, z) = AT(zv, x, y, z) + AT(sd, x, y, z);
            }
    return 0;
}

/* sd = fma(alpha, sd, beta*rt) */
int orc_tea_p2(const int64_t lo[3], const int64_t hi[3], ov sd, ov rt, double alpha, double beta)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x)
                AT(sd, x, y, z) = fma(alpha, AT(sd, x, y, z), beta * AT(rt, x, y, z));
    return 0;
}

/* rt = r; sd = r / theta; z = 0 */
int orc_tea_precon_init(const int64_t lo[3], const int64_t hi[3], ov r, ov rt, ov sd, ov zv, double theta)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double v = AT(r, x, y, z);
                AT(rt, x, y, z) = v;
                AT(sd, x, y, z) = v / theta;
                AT(zv, x, y, z) = 0.0;
            }
    return 0;
}

/* x = fma(alpha, p, x); r = fma(-alpha, w, r) */
int orc_tea_cg_update(const int64_t lo[3], const int64_t hi[3], ov xv, ov r, ov p, ov w, double alpha)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                AT(xv, x, y, z) = fma(alpha, AT(p, x, y, z), AT(xv, x, y, z));
                AT(r, x, y, z) = fma(-alpha, AT(w, x, y, z), AT(r, x, y, z));
            }
    return 0;
}

/* p = fma(beta, p, z) */
int orc_tea_cg_p(const int64_t lo[3], const int64_t hi[3], ov p, ov zv, double beta)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x)
                AT(p, x, y, z) = fma(beta, AT(p, x, y, z), AT(zv, x, y, z));
    return 0;
}

/* Gershgorin row bound 1 + 2*(sum of the cell's face coefficients), maximised. */
double orc_tea_gersh(int nd, const int64_t lo[3], const int64_t hi[3], const ov *K)
{
    double m = -INFINITY;
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double s = AT(K[0], x + 1, y, z) + AT(K[0], x, y, z);
                s = s + AT(K[1], x, y + 1, z);
                s = s + AT(K[1], x, y, z);
                if (nd == 3) {
                    s = s + AT(K[2], x, y, z + 1);
                    s = s + AT(K[2], x, y, z);
                }
                double g = fma(2.0, s, 1.0);
                if (g > m)
                    m = g;
            }
    return m;
}

/* Exact per-point products a*b as (prod, err) pairs for a dot product. */
int orc_dot_terms(const int64_t lo[3], const int64_t hi[3], ov a, ov b, double *c)
{
    int64_t i = 0;
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x, ++i) {
                double u = AT(a, x, y, z), v = AT(b, x, y, z);
                double pr = u * v;
                c[2 * i] = pr;
                c[2 * i + 1] = fma(u, v, -pr);
            }
    return 0;
}

/* ---- compressible Euler, conserved variables Q = (rho, rho u_1..rho u_D, E) ----
 * (the stand-in for the OpenSBLI Taylor-Green experiment, Section 5 and
 * Section 6.4: explicit Runge-Kutta stages of central-difference sweeps).
 *
 * Primitive variables at a point:
 *   ri = 1 / rho;  u_d = (rho u_d) * ri;
 *   k = sum over d from the last to the first of (rho u_d) u_d, accumulated
 *       as k = (rho u_D) u_D, then k = fma(rho u_d, u_d, k) for d = D-1..1;
 *   p = gm1 * fma(-0.5, k, E)              (gm1 = gamma - 1)
 * q[] holds the D + 2 conserved arrays, vel[] the D velocities. */
int orc_euler_prim(int ndim, const int64_t lo[3], const int64_t hi[3], const ov *q, const ov *vel, ov p, double gm1)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                const double ri = 1.0 / AT(q[0], x, y, z);
                double u[3];
                for (int d = 0; d < ndim; ++d) u[d] = AT(q[1 + d], x, y, z) * ri;
                double k = AT(q[ndim], x, y, z) * u[ndim - 1];
                for (int d = ndim - 2; d >= 0; --d) k = fma(AT(q[1 + d], x, y, z), u[d], k);
                for (int d = 0; d < ndim; ++d) AT(vel[d], x, y, z) = u[d];
                AT(p, x, y, z) = gm1 * fma(-0.5, k, AT(q[ndim + 1], x, y, z));
            }
    return 0;
}

/* Flux of conserved component c along axis d at a point:
 *   f = Q_c u_d;  momentum along d (c == d + 1): f = f + p;
 *   energy (c == D + 1): f = fma(p, u_d, f). */
static double euler_flux(int ndim, int c, int d, ov qc, const ov *vel, ov p, int64_t x, int64_t y, int64_t z)
{
    const double ud = AT(vel[d], x, y, z);
    double f = AT(qc, x, y, z) * ud;
    if (c == d + 1) f = f + AT(p, x, y, z);
    if (c == ndim + 1) f = fma(AT(p, x, y, z), ud, f);
    return f;
}

/* Right-hand side of component c with fourth-order central differences,
 * differences first:  for each axis d (in order), with f(o) the flux at
 * offset o along d:  t1 = f(+1) - f(-1);  t2 = f(+2) - f(-2);
 * g_d = 8 t1 - t2;  acc = g_0 (+ g_1 (+ g_2)) summed in axis order;
 * R = -acc * s   with s = 1 / (12 h). */
int orc_euler_rhs(int ndim, const int64_t lo[3], const int64_t hi[3], int c, ov r, ov qc, const ov *vel, ov p,
                  double s)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                double acc = 0.0;
                for (int d = 0; d < ndim; ++d) {
                    int64_t e[3] = {0, 0, 0};
                    e[d] = 1;
                    const double fp1 = euler_flux(ndim, c, d, qc, vel, p, x + e[0], y + e[1], z + e[2]);
                    const double fm1 = euler_flux(ndim, c, d, qc, vel, p, x - e[0], y - e[1], z - e[2]);
                    const double fp2 = euler_flux(ndim, c, d, qc, vel, p, x + 2 * e[0], y + 2 * e[1], z + 2 * e[2]);
                    const double fm2 = euler_flux(ndim, c, d, qc, vel, p, x - 2 * e[0], y - 2 * e[1], z - 2 * e[2]);
                    const double t1 = fp1 - fm1;
                    const double t2 = fp2 - fm2;
                    const double g = 8.0 * t1 - t2;
                    acc = d == 0 ? g : acc + g;
                }
                AT(r, x, y, z) = -acc * s;
            }
    return 0;
}

/* One Runge-Kutta stage of one component (Shu-Osher form):
 *   t = fma(dt, R, Q);  Q = fma(a, Q0, b t). */
int orc_rk_stage(const int64_t lo[3], const int64_t hi[3], ov q0, ov q, ov r, double a, double b, double dt)
{
    for (int64_t z = lo[2]; z < hi[2]; ++z)
        for (int64_t y = lo[1]; y < hi[1]; ++y)
            for (int64_t x = lo[0]; x < hi[0]; ++x) {
                const double t = fma(dt, AT(r, x, y, z), AT(q, x, y, z));
                AT(q, x, y, z) = fma(a, AT(q0, x, y, z), b * t);
            }
    return 0;
}

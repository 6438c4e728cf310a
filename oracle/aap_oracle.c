/*
 * Reference oracle for one time step of the metric Vicsek-class models of
 * aligning self-propelled particles (Kuersten, "Aligning Active Particles Py
 * Package", CPC).  TEST INFRASTRUCTURE ONLY: this file is the slow, plain,
 * double-precision statement of what the GPU path must compute.  Only the
 * test suite, the smoke check and the CPU baseline of the benchmark load it;
 * the product library never does, and this file shares no code with it.
 *
 * Every routine works in IEEE binary64 and is compiled without FP
 * contraction, so each comparison below is a fixed sequence of rounded
 * operations that an independent implementation can reproduce exactly.
 *
 * Paper passages followed (section / equation of the paper):
 *   - state x in [0,Lx], y in [0,Ly], theta in [-pi,pi]          Sec. 2
 *   - one VM step = collision (all theta) then streaming (all x,y) Sec. 2.1
 *   - collision rule, uniform noise eta*xi, xi ~ U[-pi,pi]        Eq. (1)
 *   - Vicsek rule f = arg[e^{i th_i} + sum_j e^{i th_j}] + omega  Eq. (2)
 *   - nematic Vicsek rule: a neighbour whose orientation differs
 *     by more than pi/2 enters turned by pi, sign(0) = +1          Eq. (3)
 *   - streaming x += v cos th(t+1), y += v sin th(t+1)            Eq. (4)
 *   - overdamped Langevin with weight h(|Omega|), order o         Eq. (5)
 *     integrated by Euler-Maruyama with Gaussian noise            Sec. 2.2
 *   - metric neighbourhood {j != i : d_ij <= R}                   Eq. (6)
 *   - periodic images (+-L) and reflecting mirror images
 *     (x -> -x or 2L-x, theta -> pi-theta), re-insertion rules    Sec. 2.4
 *   - cell lists, cells a little larger than R, 3x3 cell scan    Sec. 3.2
 *   - polar order p, mean neighbour number, moments 1..4,
 *     states t=0..n-1 of an n-step measurement                    Sec. 3.4
 *   - Binder cumulant U = 1 - <p^4>/(3<p^2>^2)                    Fig. 5
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
 *     keyed by the seed, counter (particle id, step, replica, purpose),
 *     replacing the Mersenne twister the paper uses, so that every particle's
 *     draw is addressable;  U24(w) = (w >> 8) * 2^-24;
 *   - cells per axis M = floor(L / (R (1 + 2^-20))): every cell side exceeds
 *     R by a relative margin that dominates double rounding, which makes the
 *     3x3 scan reach exactly the brute-force neighbour set, ties included;
 *   - a particle's own mirror images are not its neighbours (Eq. (6) j != i);
 *   - periodic positions live in [0,L): add L if x < 0, then subtract L if
 *     x >= L; reflecting positions in [0,L]; y-walls mirror theta -> -theta;
 *   - Langevin positions use the pre-update angle (explicit Euler-Maruyama);
 *   - arg(0) is taken as the particle's own angle.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RULE_VM 0
#define ORC_RULE_LANGEVIN 1
#define ORC_RULE_NVM 2

#define ORC_PURPOSE_NOISE_VM 0u
#define ORC_PURPOSE_NOISE_GAUSS 1u
#define ORC_PURPOSE_INIT 2u

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 bit     */
/* multiplications; the key is bumped by two Weyl constants between rounds. */
/* ------------------------------------------------------------------------ */
static const uint32_t ORC_PHILOX_M0 = 0xD2511F53u;
static const uint32_t ORC_PHILOX_M1 = 0xCD9E8D57u;
/* Weyl increments: golden ratio minus one, and sqrt(3) minus one, as 0.32 */
static const uint32_t ORC_PHILOX_W0 = 0x9E3779B9u;
static const uint32_t ORC_PHILOX_W1 = 0xBB67AE85u;

void orc_philox_constants(uint32_t out[4])
{
    out[0] = ORC_PHILOX_M0;
    out[1] = ORC_PHILOX_M1;
    out[2] = ORC_PHILOX_W0;
    out[3] = ORC_PHILOX_W1;
}

/* rounds = 10 is Philox4x32-10; other counts exist for the tests only. */
void orc_philox4x32(const uint32_t ctr_in[4], const uint32_t key_in[2],
                    int rounds, uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < rounds; ++r) {
        if (r > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void orc_draw(uint64_t seed, uint32_t id, uint64_t step,
                     uint32_t replica, uint32_t purpose, uint32_t out[4])
{
    uint32_t ctr[4] = { id, (uint32_t)step, replica, purpose };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32(ctr, key, 10, out);
}

static double orc_u24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

/* Batch access to the raw generator for the statistical tests. */
void orc_philox_batch(uint64_t seed, const uint32_t* ids, int64_t n,
                      uint64_t step, uint32_t replica, uint32_t purpose,
                      uint32_t* out /* 4 n */)
{
    for (int64_t k = 0; k < n; ++k)
        orc_draw(seed, ids[k], step, replica, purpose, out + 4 * k);
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */
int orc_cells_per_axis(double L, double R)
{
    double m = floor(L / (R * (1.0 + 0x1p-20)));
    if (m < 1.0) return 0;
    if (m > 2147483647.0) return 2147483647;
    return (int)m;
}

static double orc_wrap_angle(double th)
{
    const double two_pi = 2.0 * M_PI;
    double w = th - two_pi * floor((th + M_PI) / two_pi);
    if (w >= M_PI) w -= two_pi;
    if (w < -M_PI) w += two_pi;
    return w;
}

double orc_wrap_angle_export(double th) { return orc_wrap_angle(th); }

static int orc_cell_of(double x, double invcs, int M)
{
    double u = x * invcs;
    int64_t c = (int64_t)u;       /* truncation == floor for u >= 0 */
    if (u < 0.0) c = 0;
    if (c > M - 1) c = M - 1;
    return (int)c;
}

/* Cell key = cy * Mx + cx (row-major), the bin of the cell lists. */
void orc_cell_keys(int64_t N, const double* x, const double* y,
                   double Lx, double Ly, double R, uint32_t* key)
{
    int Mx = orc_cells_per_axis(Lx, R), My = orc_cells_per_axis(Ly, R);
    double ix = (double)Mx / Lx, iy = (double)My / Ly;
    for (int64_t i = 0; i < N; ++i) {
        int cx = orc_cell_of(x[i], ix, Mx);
        int cy = orc_cell_of(y[i], iy, My);
        key[i] = (uint32_t)((int64_t)cy * Mx + cx);
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbour sums                                                           */
/* ------------------------------------------------------------------------ */
/*
 * sign(cos(th_i - th~_j)) of Eq. (3), with sign(0) = +1, where th~_j is the
 * orientation of the image of j: th_j, pi - th_j (x mirror), -th_j (y mirror)
 * or th_j - pi (both mirrors).
 *
 * By cos(a - pi) = -cos(a), cos(th_i - th~_j) = sigma cos(s) with
 *   s = th_i - th_j, sigma = +1   (no mirror)
 *   s = th_i + th_j, sigma = -1   (x mirror)
 *   s = th_i + th_j, sigma = +1   (y mirror)
 *   s = th_i - th_j, sigma = -1   (both).
 * s is formed with one binary64 rounding and, for |s| < 5 pi / 2,
 * cos(s) > 0 exactly when |s| < pi/2 or |s| > 3 pi/2.  The comparisons use
 * PI_2_DN, the largest binary64 below pi/2, and PI3_2_UP, the smallest
 * binary64 above 3 pi/2: for a binary64 s they decide |s| < pi/2 and
 * |s| > 3 pi/2 without error.  With binary32 angles of magnitude >= 2^-28
 * (and at most pi in binary32) s is exact, so the sign is that of exact
 * arithmetic on the given angles; a smaller angle leaves s within 2^-51 of
 * its exact value but at least 4e-8 away from every zero of cos (no
 * binary32 number lies closer than 4.3e-8 to pi/2), so again the sign is
 * exact.  cos(s) = 0 cannot occur for s a nonzero binary64.
 */
static const double ORC_PI_2_DN = 0x1.921fb54442d18p+0;
static const double ORC_PI3_2_UP = 0x1.2d97c7f3321d3p+2;

int orc_nvm_sign(double thi, double thj, int mirror_x, int mirror_y)
{
    const double s = (mirror_x != mirror_y) ? thi + thj : thi - thj;
    const double as = fabs(s);
    const int cos_pos = (as <= ORC_PI_2_DN) || (as >= ORC_PI3_2_UP);
    const int sigma = mirror_x ? -1 : 1;
    return cos_pos ? sigma : -sigma;
}

/*
 * One candidate image of particle j as seen by particle i.
 *   periodic axis:   image x = x_j + s with s in {-L, 0, +L}
 *   reflecting axis: image x = x_j, -x_j (wall x=0) or 2L - x_j (wall x=L)
 * The mirrored orientation is theta -> pi - theta for a vertical wall and
 * theta -> -theta for a horizontal wall; both compose at corners.
 */
static void orc_accumulate(double xi, double yi, double thi,
                           double ximg, double yimg, double thj,
                           int mirror_x, int mirror_y, double R2, int rule, int order,
                           int64_t* n, double* C, double* S, double* A)
{
    double dx = ximg - xi;
    double dy = yimg - yi;
    double d2 = dx * dx + dy * dy;
    if (!(d2 <= R2)) return;
    double t = thj;
    if (mirror_x) t = M_PI - t;
    if (mirror_y) t = -t;
    *n += 1;
    if (rule == ORC_RULE_NVM) {
        /* Eq. (3): the term exp[i (th~_j + pi/2 (1 - sign(cos(th_i - th~_j))))] */
        const double sg = (double)orc_nvm_sign(thi, thj, mirror_x, mirror_y);
        const double ph = t + M_PI_2 * (1.0 - sg);
        *C += cos(ph);
        *S += sin(ph);
    } else {
        *C += cos(t);
        *S += sin(t);
    }
    *A += sin((double)order * (t - thi));
}

/*
 * Brute force over every particle and every image: the definition of Eq. (6)
 * with the images of Sec. 2.4 written out.  For each i in idx[0..nidx):
 *   n[k] = |Omega_i|,
 *   C[k] + i S[k] = e^{i th_i} + sum_{Omega_i} e^{i th~_j}   (Eq. (2) bracket;
 *                   for the NVM the bracket of Eq. (3))
 *   A[k] = sum_{Omega_i} sin(o (th~_j - th_i))              (Eq. (5) sum)
 */
void orc_neighbours_brute(int64_t N, const double* x, const double* y,
                          const double* th, double Lx, double Ly, double R,
                          int bx, int by, int rule, int order,
                          const int64_t* idx, int64_t nidx,
                          int64_t* n_out, double* C_out, double* S_out,
                          double* A_out)
{
    const double R2 = R * R;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nidx; ++k) {
        int64_t i = idx[k];
        double xi = x[i], yi = y[i], thi = th[i];
        int64_t n = 0;
        double C = cos(thi), S = sin(thi), A = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double xs[3], ys[3];
            int mxs[3], mys[3];
            if (bx) {
                xs[0] = x[j];        mxs[0] = 0;
                xs[1] = -x[j];       mxs[1] = 1;
                xs[2] = 2.0 * Lx - x[j]; mxs[2] = 1;
            } else {
                xs[0] = x[j] + (-Lx); mxs[0] = 0;
                xs[1] = x[j];         mxs[1] = 0;
                xs[2] = x[j] + Lx;    mxs[2] = 0;
            }
            if (by) {
                ys[0] = y[j];        mys[0] = 0;
                ys[1] = -y[j];       mys[1] = 1;
                ys[2] = 2.0 * Ly - y[j]; mys[2] = 1;
            } else {
                ys[0] = y[j] + (-Ly); mys[0] = 0;
                ys[1] = y[j];         mys[1] = 0;
                ys[2] = y[j] + Ly;    mys[2] = 0;
            }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    orc_accumulate(xi, yi, thi, xs[a], ys[b], th[j],
                                   mxs[a], mys[b], R2, rule, order, &n, &C, &S, &A);
        }
        n_out[k] = n;
        C_out[k] = C;
        S_out[k] = S;
        A_out[k] = A;
    }
}

/*
 * Cell lists as in Sec. 3.2: one list per cell, rebuilt on every call; the
 * neighbours of i are searched in its own and the eight surrounding cells.
 * Virtual cells beyond a periodic edge are the wrapped cells shifted by L;
 * beyond a reflecting edge they are the mirror images of the edge cells.
 */
void orc_neighbours_cells(int64_t N, const double* x, const double* y,
                          const double* th, double Lx, double Ly, double R,
                          int bx, int by, int rule, int order,
                          int64_t* n_out, double* C_out, double* S_out,
                          double* A_out)
{
    const int Mx = orc_cells_per_axis(Lx, R), My = orc_cells_per_axis(Ly, R);
    const double R2 = R * R;
    const double ix = (double)Mx / Lx, iy = (double)My / Ly;
    int64_t ncell = (int64_t)Mx * My;
    int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int* cxs = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int* cys = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
    for (int64_t i = N - 1; i >= 0; --i) {
        cxs[i] = orc_cell_of(x[i], ix, Mx);
        cys[i] = orc_cell_of(y[i], iy, My);
        int64_t c = (int64_t)cys[i] * Mx + cxs[i];
        next[i] = head[c];
        head[c] = i;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        double xi = x[i], yi = y[i], thi = th[i];
        int64_t n = 0;
        double C = cos(thi), S = sin(thi), A = 0.0;
        for (int dcy = -1; dcy <= 1; ++dcy) {
            int vy = cys[i] + dcy;
            int gy = vy;
            int ymode = 0;      /* 0 identity, 1 shift -L, 2 shift +L, 3 mirror 0, 4 mirror L */
            if (vy < 0) {
                if (by) { gy = 0; ymode = 3; } else { gy = My - 1; ymode = 1; }
            } else if (vy >= My) {
                if (by) { gy = My - 1; ymode = 4; } else { gy = 0; ymode = 2; }
            }
            for (int dcx = -1; dcx <= 1; ++dcx) {
                int vx = cxs[i] + dcx;
                int gx = vx;
                int xmode = 0;
                if (vx < 0) {
                    if (bx) { gx = 0; xmode = 3; } else { gx = Mx - 1; xmode = 1; }
                } else if (vx >= Mx) {
                    if (bx) { gx = Mx - 1; xmode = 4; } else { gx = 0; xmode = 2; }
                }
                for (int64_t j = head[(int64_t)gy * Mx + gx]; j >= 0; j = next[j]) {
                    if (j == i) continue;
                    double ximg, yimg;
                    switch (xmode) {
                    case 1: ximg = x[j] + (-Lx); break;
                    case 2: ximg = x[j] + Lx; break;
                    case 3: ximg = -x[j]; break;
                    case 4: ximg = 2.0 * Lx - x[j]; break;
                    default: ximg = x[j]; break;
                    }
                    switch (ymode) {
                    case 1: yimg = y[j] + (-Ly); break;
                    case 2: yimg = y[j] + Ly; break;
                    case 3: yimg = -y[j]; break;
                    case 4: yimg = 2.0 * Ly - y[j]; break;
                    default: yimg = y[j]; break;
                    }
                    orc_accumulate(xi, yi, thi, ximg, yimg, th[j],
                                   xmode >= 3, ymode >= 3, R2, rule, order,
                                   &n, &C, &S, &A);
                }
            }
        }
        n_out[i] = n;
        C_out[i] = C;
        S_out[i] = S;
        A_out[i] = A;
    }
    free(head);
    free(next);
    free(cxs);
    free(cys);
}

/* ------------------------------------------------------------------------ */
/* Re-insertion into the box (Sec. 2.4)                                     */
/* ------------------------------------------------------------------------ */
static void orc_boundary(double* x, double* y, double* th,
                         double Lx, double Ly, int bx, int by)
{
    if (bx) {
        if (*x < 0.0) { *x = -*x; *th = M_PI - *th; }
        else if (*x > Lx) { *x = 2.0 * Lx - *x; *th = M_PI - *th; }
    } else {
        if (*x < 0.0) *x += Lx;
        if (*x >= Lx) *x -= Lx;
    }
    if (by) {
        if (*y < 0.0) { *y = -*y; *th = -*th; }
        else if (*y > Ly) { *y = 2.0 * Ly - *y; *th = -*th; }
    } else {
        if (*y < 0.0) *y += Ly;
        if (*y >= Ly) *y -= Ly;
    }
    *th = orc_wrap_angle(*th);
}

/* ------------------------------------------------------------------------ */
/* Update rules                                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    double Lx, Ly, R, v, eta, omega, gamma, dt;
    int rule, order, bx, by;
    uint64_t seed;
    const double* weights;
    int weight_len;
    uint32_t replica;   /* counter word 2: independent streams of one seed */
} orc_params;

/* Uniform noise xi in [-pi, pi] of Eq. (1) for particle id at step t. */
static double orc_noise_vm_r(uint64_t seed, uint32_t id, uint64_t t, uint32_t replica)
{
    uint32_t w[4];
    orc_draw(seed, id, t, replica, ORC_PURPOSE_NOISE_VM, w);
    double u = orc_u24(w[0]);
    return M_PI * (2.0 * u - 1.0);
}

/* Standard Gaussian by Box-Muller (Sec. 3.1), cosine branch. */
static double orc_noise_gauss_r(uint64_t seed, uint32_t id, uint64_t t, uint32_t replica)
{
    uint32_t w[4];
    orc_draw(seed, id, t, replica, ORC_PURPOSE_NOISE_GAUSS, w);
    double u1 = ((double)(w[0] >> 8) + 1.0) * 0x1p-24;   /* (0, 1] */
    double u2 = (double)(w[1] >> 8) * 0x1p-24;           /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

double orc_noise_vm(uint64_t seed, uint32_t id, uint64_t t)
{
    return orc_noise_vm_r(seed, id, t, 0u);
}

double orc_noise_gauss(uint64_t seed, uint32_t id, uint64_t t)
{
    return orc_noise_gauss_r(seed, id, t, 0u);
}

static double orc_weight(const orc_params* p, int64_t n)
{
    if (!p->weights || p->weight_len < 1) return 1.0;
    int64_t k = n < p->weight_len - 1 ? n : p->weight_len - 1;
    return p->weights[k];
}

/*
 * Update every particle from its neighbour sums (state t -> t+1).
 * th_in/x_in/y_in are the state at time t; outputs may alias inputs.
 */
void orc_update(int64_t N, const orc_params* p, uint64_t t,
                const uint32_t* ids, const double* x, const double* y,
                const double* th, const int64_t* n, const double* C,
                const double* S, const double* A,
                double* x_out, double* y_out, double* th_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double xn, yn, tn;
        if (p->rule != ORC_RULE_LANGEVIN) {
            /* Eq. (1) with Eq. (2) (VM) or Eq. (3) (NVM; C, S carry its
               bracket): collision, then Eq. (4): streaming with th(t+1) */
            double f = (C[i] == 0.0 && S[i] == 0.0) ? th[i] : atan2(S[i], C[i]);
            tn = f + p->omega + p->eta * orc_noise_vm_r(p->seed, ids[i], t, p->replica);
            tn = orc_wrap_angle(tn);
            xn = x[i] + p->v * cos(tn);
            yn = y[i] + p->v * sin(tn);
        } else {
            /* Eq. (5) by Euler-Maruyama: positions with th(t) */
            double g = orc_noise_gauss_r(p->seed, ids[i], t, p->replica);
            double drift = p->gamma * orc_weight(p, n[i]) * A[i] + p->omega;
            tn = th[i] + p->dt * drift + p->eta * sqrt(p->dt) * g;
            xn = x[i] + p->v * p->dt * cos(th[i]);
            yn = y[i] + p->v * p->dt * sin(th[i]);
        }
        orc_boundary(&xn, &yn, &tn, p->Lx, p->Ly, p->bx, p->by);
        x_out[i] = xn;
        y_out[i] = yn;
        th_out[i] = tn;
    }
}

/* ------------------------------------------------------------------------ */
/* Initial state: uniform positions, isotropic orientations (Sec. 5)        */
/* ------------------------------------------------------------------------ */
void orc_init(int64_t N, double Lx, double Ly, int bx, int by, uint64_t seed,
              uint32_t replica, double* x, double* y, double* th)
{
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        orc_draw(seed, (uint32_t)i, 0u, replica, ORC_PURPOSE_INIT, w);
        double xx = Lx * orc_u24(w[0]);
        double yy = Ly * orc_u24(w[1]);
        double tt = M_PI * (2.0 * orc_u24(w[2]) - 1.0);
        if (!bx && xx >= Lx) xx -= Lx;
        if (!by && yy >= Ly) yy -= Ly;
        x[i] = xx;
        y[i] = yy;
        th[i] = tt;
    }
}

/* ------------------------------------------------------------------------ */
/* Measurement of one state (Sec. 3.4): p and the mean neighbour number     */
/* ------------------------------------------------------------------------ */
/*
 * Order parameters of one state (Sec. 3.4): polar p = |sum e^{i th}| / N,
 * nematic q = |sum e^{2 i th}| / N, and nbar = sum n / N.  q_out may be NULL.
 */
void orc_state_observables(int64_t N, const double* th, const int64_t* n,
                           double* p_out, double* nbar_out, double* q_out)
{
    double sc = 0.0, ss = 0.0, sn = 0.0, sc2 = 0.0, ss2 = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        sc += cos(th[i]);
        ss += sin(th[i]);
        sc2 += cos(2.0 * th[i]);
        ss2 += sin(2.0 * th[i]);
        sn += (double)n[i];
    }
    *p_out = sqrt(sc * sc + ss * ss) / (double)N;
    *nbar_out = sn / (double)N;
    if (q_out) *q_out = sqrt(sc2 * sc2 + ss2 * ss2) / (double)N;
}

/*
 * Adds one state to the histograms of the angles and of the neighbour
 * numbers (Sec. 3.4).  Angle bin k covers [-pi + 2 pi k / bt,
 * -pi + 2 pi (k+1) / bt); the bin of an angle is floor((th + pi) * (bt / (2 pi)))
 * in binary64 (pi the binary64 value nearest to it), clamped to [0, bt-1].
 * Neighbour numbers n >= bn - 1 fall in the last bin.
 */
void orc_histograms(int64_t N, const double* th, const int64_t* n, int bt, int bn,
                    int64_t* ht, int64_t* hn)
{
    const double pi = 3.14159265358979311600;
    const double scale = (double)bt / (2.0 * pi);
    for (int64_t i = 0; i < N; ++i) {
        const double u = (th[i] + pi) * scale;
        int64_t k = 0;
        if (u >= (double)bt) k = bt - 1;
        else if (u > 0.0) k = (int64_t)u;
        ht[k] += 1;
        const int64_t m = n[i] < bn - 1 ? n[i] : bn - 1;
        hn[m] += 1;
    }
}

/*
 * nsteps full steps with cell lists, in physics mode (double state).
 * State arrays are indexed by particle id.  When measure != 0 the states
 * t0 .. t0+nsteps-1 are measured (Sec. 3.4): p_series[k], nbar_series[k]
 * and q_series[k] receive p, nbar and q of state t0+k (any may be NULL);
 * when ht and hn are given, each measured state is added to the histograms
 * (bt angle bins, bn neighbour bins).
 */
int orc_run(int64_t N, const orc_params* p, uint64_t t0, int64_t nsteps,
            double* x, double* y, double* th,
            double* p_series, double* nbar_series, double* q_series,
            int bt, int bn, int64_t* ht, int64_t* hn)
{
    int64_t* n = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    double* C = (double*)malloc(sizeof(double) * (size_t)N);
    double* S = (double*)malloc(sizeof(double) * (size_t)N);
    double* A = (double*)malloc(sizeof(double) * (size_t)N);
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
    if (!n || !C || !S || !A || !ids) {
        free(n); free(C); free(S); free(A); free(ids);
        return -2;
    }
    for (int64_t i = 0; i < N; ++i) ids[i] = (uint32_t)i;
    for (int64_t k = 0; k < nsteps; ++k) {
        orc_neighbours_cells(N, x, y, th, p->Lx, p->Ly, p->R, p->bx, p->by,
                             p->rule, p->order, n, C, S, A);
        if (p_series || nbar_series || q_series) {
            double pv, nv, qv;
            orc_state_observables(N, th, n, &pv, &nv, &qv);
            if (p_series) p_series[k] = pv;
            if (nbar_series) nbar_series[k] = nv;
            if (q_series) q_series[k] = qv;
        }
        if (ht && hn) orc_histograms(N, th, n, bt, bn, ht, hn);
        orc_update(N, p, t0 + (uint64_t)k, ids, x, y, th, n, C, S, A, x, y, th);
    }
    free(n); free(C); free(S); free(A); free(ids);
    return 0;
}

/* Thread count of the OpenMP loops above (timing only: every result is
 * independent of it, since each particle's work and draws are its own). */
#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int n) { (void)n; }
int orc_max_threads(void) { return 1; }
#endif

/*
 * FP64 CPU oracle for the MRS filament hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It is a plain, slow, obviously correct restatement of the
 * paper's definitions (arxiv 2604.12083), in double precision, written so a
 * reader can check each function against the cited passage by eye:
 *
 *   - blob function                       Sec. II.C (blob equation)
 *   - kernel functions H1..H5             Sec. II.C, Eqs. velocity_field and
 *                                         angular_velocity_field; the paper
 *                                         names them without printing them,
 *                                         so they are the closed forms of the
 *                                         regularised Stokeslet, rotlet and
 *                                         potential dipole of this blob
 *   - direct superposition sum            Sec. II.C, Eq. superposition
 *   - rotation square root                Sec. III.B.1, Eqs. rodrigues and
 *                                         halfangle (principal root)
 *   - literal paper square-root routine   Sec. III.B.1 (for the accuracy
 *                                         protocol of Table II only)
 *   - discrete rod forces and torques     Sec. II.B, Eqs. discrete_f,
 *                                         discrete_n, F_comp_discrete,
 *                                         N_comp_discrete, mid_triad; Alg. 1
 *   - Rodrigues frame update              Sec. III.B.3, Eqs. newx, newD
 *   - RK4 stage scheme                    Sec. III.A (fine propagator is an
 *                                         explicit Runge-Kutta method)
 *   - swimming waveform                   Sec. IV (preferred strain-twist
 *                                         vector (0, -k^2 A sin(ks + ft), 0))
 *   - Lennard-Jones repulsion             Sec. IV (potential 4e((s/r)^12 -
 *                                         (s/r)^6) below r_c = 2^(1/6) s)
 *
 * Layouts: positions, forces, torques, velocities are row-major n x 3.
 * Frames are n x 9 with D[9k + 3i + c] = component c of director D^{i+1}
 * at point k.  Filaments are concatenated and delimited by CSR offsets.
 *
 * The sums over sources run in source order j = 0..N-1 for every target.
 * OpenMP only distributes independent targets over threads; it does not
 * change any target's arithmetic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Blob function of Sec. II.C: phi_eps(r) = 15 eps^4 / (8 pi (r^2 + eps^2)^{7/2}). */
double oracle_blob(double r, double eps) {
    double R2 = r * r + eps * eps;
    return 15.0 * pow(eps, 4) / (8.0 * PI * pow(R2, 3.5));
}

/*
 * Kernel functions H1..H5 of Eqs. velocity_field / angular_velocity_field
 * for the blob of Sec. II.C, with R = sqrt(r^2 + eps^2):
 *   H1 = (r^2 + 2 eps^2) / (8 pi R^3)         regularised Stokeslet, identity part
 *   H2 = 1 / (8 pi R^3)                       regularised Stokeslet, r r^T part
 *   H3 = (2 r^2 + 5 eps^2) / (16 pi R^5)      regularised rotlet
 *   H4 = (10 eps^4 - 7 eps^2 r^2 - 2 r^4) / (32 pi R^7)
 *   H5 = 3 (2 r^2 + 7 eps^2) / (32 pi R^7)    blob term plus regularised
 *                                             potential dipole
 * They follow from phi_eps by the regularised-Stokeslet construction
 * (Delta G = phi, Delta B = G, torque as the body force curl(n phi)/2,
 * omega = curl(u)/2); the tests re-derive them symbolically from the blob.
 */
void oracle_hfuncs(double r, double eps, double *H) {
    double r2 = r * r, e2 = eps * eps;
    double R = sqrt(r2 + e2);
    double R3 = R * R * R, R5 = R3 * R * R, R7 = R5 * R * R;
    H[0] = (r2 + 2.0 * e2) / (8.0 * PI * R3);
    H[1] = 1.0 / (8.0 * PI * R3);
    H[2] = (2.0 * r2 + 5.0 * e2) / (16.0 * PI * R5);
    H[3] = (10.0 * e2 * e2 - 7.0 * e2 * r2 - 2.0 * r2 * r2) / (32.0 * PI * R7);
    H[4] = 3.0 * (2.0 * r2 + 7.0 * e2) / (32.0 * PI * R7);
}

/*
 * Velocity U and angular velocity W at nt arbitrary targets xt induced by
 * ns point forces f and torques tq at X (Eqs. velocity_field,
 * angular_velocity_field summed by Eq. superposition), r = x_i - X_j:
 *   mu U_i = sum_j H1 f_j + H2 (f_j . r) r + H3 (n_j x r)
 *   mu W_i = sum_j H3 (f_j x r) + H4 n_j + H5 (n_j . r) r
 */
void oracle_mrs_field(int64_t nt, const double *xt, int64_t ns, const double *X,
                      const double *f, const double *tq, double eps, double mu,
                      double *U, double *W) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < nt; i++) {
        double u[3] = {0.0, 0.0, 0.0}, w[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < ns; j++) {
            const double *fj = f + 3 * j, *nj = tq + 3 * j;
            double r[3] = {xt[3 * i] - X[3 * j], xt[3 * i + 1] - X[3 * j + 1], xt[3 * i + 2] - X[3 * j + 2]};
            double H[5];
            oracle_hfuncs(sqrt(dot3(r, r)), eps, H);
            double fr = dot3(fj, r), nr = dot3(nj, r);
            double nxr[3], fxr[3];
            cross3(nj, r, nxr);
            cross3(fj, r, fxr);
            for (int c = 0; c < 3; c++) {
                u[c] += H[0] * fj[c] + H[1] * fr * r[c] + H[2] * nxr[c];
                w[c] += H[2] * fxr[c] + H[3] * nj[c] + H[4] * nr * r[c];
            }
        }
        for (int c = 0; c < 3; c++) {
            U[3 * i + c] = u[c] / mu;
            W[3 * i + c] = w[c] / mu;
        }
    }
}

/* Eq. superposition with the targets being the sources themselves (j = i included). */
void oracle_mrs_eval(int64_t n, const double *X, const double *f, const double *tq,
                     double eps, double mu, double *U, double *W) {
    oracle_mrs_field(n, X, n, X, f, tq, eps, mu, U, W);
}

/* ---------------------------------------------------------------------- */
/* 3x3 rotations.  Matrices are row-major: M[3*row + col].                 */

/* Eq. halfangle / Eq. rodrigues: rotation by angle t about unit axis n. */
static void axis_angle_matrix(const double *n, double t, double *S) {
    double c = cos(t), s = sin(t);
    double K[9] = {0.0, -n[2], n[1], n[2], 0.0, -n[0], -n[1], n[0], 0.0};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            S[3 * i + j] = (i == j ? c : 0.0) + (1.0 - c) * n[i] * n[j] + s * K[3 * i + j];
}

/*
 * Axis n and angle theta in [0, pi] of a proper rotation R (Eq. rodrigues).
 * cos(theta) = (tr R - 1)/2 and the skew part gives 2 sin(theta) n.  Where
 * sin(theta) is small and cos(theta) < 0 (theta near pi) the skew part no
 * longer fixes n accurately, so n is read from the symmetric part
 * R + R^T - 2 cos(theta) I = 2 (1 - cos(theta)) n n^T instead, with its sign
 * taken from the skew part.
 */
static void rotation_axis_angle(const double *R, double *n, double *theta) {
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]}; /* 2 sin(theta) n */
    double s = 0.5 * sqrt(dot3(v, v));
    *theta = atan2(s, c);
    if (s == 0.0 && c > 0.0) { /* identity: any axis */
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
        return;
    }
    if (c >= -0.5) {
        for (int k = 0; k < 3; k++) n[k] = v[k] / (2.0 * s);
    } else {
        double P[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++)
                P[3 * i + j] = (R[3 * i + j] + R[3 * j + i] - (i == j ? 2.0 * c : 0.0)) / (2.0 * (1.0 - c));
        int k = 0;
        if (P[4] > P[3 * k + k]) k = 1;
        if (P[8] > P[3 * k + k]) k = 2;
        double len = sqrt(P[3 * k + k]);
        for (int i = 0; i < 3; i++) n[i] = P[3 * i + k] / len;
        if (dot3(n, v) < 0.0)
            for (int i = 0; i < 3; i++) n[i] = -n[i];
        double nn = sqrt(dot3(n, n));
        for (int i = 0; i < 3; i++) n[i] /= nn;
    }
}

/* Principal square root of a rotation: the rotation about the same axis by
 * half the angle (Eq. halfangle). */
void oracle_rotsqrt(const double *R, double *S) {
    double n[3], theta;
    rotation_axis_angle(R, n, &theta);
    axis_angle_matrix(n, 0.5 * theta, S);
}

void oracle_rotsqrt_batch(int64_t count, const double *R, double *S) {
    for (int64_t i = 0; i < count; i++) oracle_rotsqrt(R + 9 * i, S + 9 * i);
}

/*
 * The square-root routine exactly as Sec. III.B.1 describes it, for the
 * accuracy protocol of Table II: cos(theta) from the trace; S = I when
 * theta < tol0; when pi - theta < tolpi the axis comes from the diagonal,
 * n_i^2 = (R_ii + 1)/2, and S = R(pi/2, n); otherwise the axis comes from
 * the skew part divided by 2 sin(theta) and S is Eq. halfangle.  The paper
 * fixes neither threshold nor the signs of the diagonal axis; the signs are
 * taken relative to the largest component from the off-diagonal sums.
 */
void oracle_rotsqrt_literal(const double *R, double *S, double tol0, double tolpi) {
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double theta = acos(c);
    double n[3];
    if (theta < tol0) {
        for (int i = 0; i < 9; i++) S[i] = (i % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    if (PI - theta < tolpi) {
        for (int i = 0; i < 3; i++) {
            double q = 0.5 * (R[4 * i] + 1.0);
            n[i] = sqrt(q > 0.0 ? q : 0.0);
        }
        int k = 0;
        if (n[1] > n[k]) k = 1;
        if (n[2] > n[k]) k = 2;
        for (int i = 0; i < 3; i++)
            if (i != k && R[3 * i + k] + R[3 * k + i] < 0.0) n[i] = -n[i];
        axis_angle_matrix(n, 0.5 * PI, S);
        return;
    }
    double s = sin(theta);
    n[0] = (R[7] - R[5]) / (2.0 * s);
    n[1] = (R[2] - R[6]) / (2.0 * s);
    n[2] = (R[3] - R[1]) / (2.0 * s);
    axis_angle_matrix(n, 0.5 * theta, S);
}

/* Eq. newD: v = omega dt, theta = |v|, e = v/|v|;
 * D' = cos(theta) D + sin(theta) (e x D) + (1 - cos(theta)) (e . D) e. */
void oracle_rodrigues(const double *v, const double *D, double *out) {
    double theta = sqrt(dot3(v, v));
    if (theta == 0.0) {
        out[0] = D[0]; out[1] = D[1]; out[2] = D[2];
        return;
    }
    double e[3] = {v[0] / theta, v[1] / theta, v[2] / theta};
    double exD[3];
    cross3(e, D, exD);
    double eD = dot3(e, D), c = cos(theta), s = sin(theta);
    double o[3];
    for (int k = 0; k < 3; k++) o[k] = c * D[k] + s * exD[k] + (1.0 - c) * eD * e[k];
    out[0] = o[0]; out[1] = o[1]; out[2] = o[2];
}

/* ---------------------------------------------------------------------- */
/* Discrete Kirchhoff rod (Sec. II.B, Alg. 1).                             */

/*
 * Point force g_k and torque m_k exerted on the fluid by each node.
 *
 * Per segment k+1/2 (nodes k, k+1 of one filament):
 *   A = sum_j D^j_{k+1} (D^j_k)^T, D^i_h = A^{1/2} D^i_k        (Eq. mid_triad)
 *   F^j = b_j ((X_{k+1} - X_k)/ds . D^j_h - delta_3j)          (Eq. F_comp_discrete)
 *   N^i = a_i ((D^j_{k+1} - D^j_k)/ds . D^l_h - Omega_i),
 *         (i, j, l) a cyclic permutation of (1, 2, 3)          (Eq. N_comp_discrete)
 *   F = sum_j F^j D^j_h, N = sum_i N^i D^i_h
 * Per node, with F, N of absent end segments equal to zero (free ends):
 *   f_k = -(F_{k+1/2} - F_{k-1/2})/ds                            (Eq. discrete_f)
 *   n_k = -(N_{k+1/2} - N_{k-1/2})/ds
 *         - (dX_{k+1/2}/ds x F_{k+1/2} + dX_{k-1/2}/ds x F_{k-1/2})/2   (Eq. discrete_n)
 * f_k, n_k are densities exerted by the fluid on the rod (Sec. II.A), so the
 * point force and torque the node exerts on the fluid are -ds f_k and
 * -ds n_k; the external point loads fext, next are added to them.
 */
/*
 * Swimming (Sec. IV): with wave = (A, k, f), the preferred strain-twist
 * vector of segment k+1/2 at time t is om0 + (0, -k^2 A sin(k s + f t), 0)
 * with s = (k + 1/2) ds its arclength, the segment midpoint.
 */
static void preferred_strain(const double *om0, const double *wave, double t, double s, double *om) {
    om[0] = om0[0];
    om[1] = om0[1];
    om[2] = om0[2];
    if (wave) om[1] += -wave[1] * wave[1] * wave[0] * sin(wave[1] * s + wave[2] * t);
}

/*
 * Lennard-Jones repulsion between points of different filaments (Sec. IV):
 * U(r) = 4 e ((sig/r)^12 - (sig/r)^6) for r < r_c = 2^(1/6) sig, zero beyond,
 * lj = (sig, e).  The force on point j is -grad_j of the pair energies,
 *   F_j = sum_i 24 e (2 (sig/r)^12 - (sig/r)^6) (x_j - x_i) / r^2,
 * over points i of other filaments with r = |x_j - x_i| < r_c.  It is a force
 * on the rod point, which a massless point passes on to the fluid, so it is
 * added to the point force on the fluid like an external load.
 */
void oracle_lj_forces(int32_t nfil, const int32_t *off, const double *X, const double *lj, double *F) {
    const int64_t n = off[nfil];
    const double sig = lj[0], e = lj[1], rc = pow(2.0, 1.0 / 6.0) * sig;
    int32_t *fil = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t fi = 0; fi < nfil; fi++)
        for (int32_t k = off[fi]; k < off[fi + 1]; k++) fil[k] = fi;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; j++) {
        double acc[3] = {0, 0, 0};
        for (int64_t i = 0; i < n; i++) {
            if (fil[i] == fil[j]) continue;
            double r[3] = {X[3 * j] - X[3 * i], X[3 * j + 1] - X[3 * i + 1], X[3 * j + 2] - X[3 * i + 2]};
            double r2 = dot3(r, r), rr = sqrt(r2);
            if (rr >= rc) continue;
            double s6 = pow(sig / rr, 6.0);
            double c = 24.0 * e * (2.0 * s6 * s6 - s6) / r2;
            for (int q = 0; q < 3; q++) acc[q] += c * r[q];
        }
        for (int q = 0; q < 3; q++) F[3 * j + q] = acc[q];
    }
    free(fil);
}

/* Total Lennard-Jones energy, each pair of points of different filaments once. */
double oracle_lj_energy(int32_t nfil, const int32_t *off, const double *X, const double *lj) {
    const double sig = lj[0], e = lj[1], rc = pow(2.0, 1.0 / 6.0) * sig;
    double E = 0.0;
    for (int32_t fa = 0; fa < nfil; fa++)
        for (int32_t fb = fa + 1; fb < nfil; fb++)
            for (int32_t i = off[fa]; i < off[fa + 1]; i++)
                for (int32_t j = off[fb]; j < off[fb + 1]; j++) {
                    double r[3] = {X[3 * j] - X[3 * i], X[3 * j + 1] - X[3 * i + 1], X[3 * j + 2] - X[3 * i + 2]};
                    double rr = sqrt(dot3(r, r));
                    if (rr >= rc) continue;
                    double s6 = pow(sig / rr, 6.0);
                    E += 4.0 * e * (s6 * s6 - s6);
                }
    return E;
}

/* oracle_rod_forces with the swimming waveform at time t (wave may be NULL)
 * and the Lennard-Jones repulsion (lj may be NULL). */
void oracle_rod_forces_ex(int32_t nfil, const int32_t *off, const double *X, const double *D,
                          const double *a, const double *b, const double *om0, double ds,
                          const double *fext, const double *next, const double *wave, double t,
                          const double *lj, double *g, double *m) {
    for (int32_t fi = 0; fi < nfil; fi++) {
        int32_t k0 = off[fi], M = off[fi + 1] - off[fi];
        int32_t nseg = M > 1 ? M - 1 : 0;
        double *Fs = calloc((size_t)(3 * (nseg + 1)), sizeof(double));
        double *Ns = calloc((size_t)(3 * (nseg + 1)), sizeof(double));
        double *dXs = calloc((size_t)(3 * (nseg + 1)), sizeof(double));
        for (int32_t k = 0; k < nseg; k++) {
            const double *Dk = D + 9 * (k0 + k), *Dk1 = D + 9 * (k0 + k + 1);
            double A[9] = {0}, S[9], Dh[9];
            for (int j = 0; j < 3; j++)
                for (int r = 0; r < 3; r++)
                    for (int c = 0; c < 3; c++) A[3 * r + c] += Dk1[3 * j + r] * Dk[3 * j + c];
            oracle_rotsqrt(A, S);
            for (int i = 0; i < 3; i++)
                for (int r = 0; r < 3; r++) {
                    double s = 0.0;
                    for (int c = 0; c < 3; c++) s += S[3 * r + c] * Dk[3 * i + c];
                    Dh[3 * i + r] = s;
                }
            double dX[3];
            for (int c = 0; c < 3; c++) dX[c] = X[3 * (k0 + k + 1) + c] - X[3 * (k0 + k) + c];
            double F[3] = {0, 0, 0}, Nv[3] = {0, 0, 0};
            for (int j = 0; j < 3; j++) {
                double Fj = b[j] * ((dX[0] * Dh[3 * j] + dX[1] * Dh[3 * j + 1] + dX[2] * Dh[3 * j + 2]) / ds -
                                    (j == 2 ? 1.0 : 0.0));
                for (int c = 0; c < 3; c++) F[c] += Fj * Dh[3 * j + c];
            }
            double om[3];
            preferred_strain(om0, wave, t, (k + 0.5) * ds, om);
            for (int i = 0; i < 3; i++) {
                int j = (i + 1) % 3, l = (i + 2) % 3;
                double dd[3];
                for (int c = 0; c < 3; c++) dd[c] = (Dk1[3 * j + c] - Dk[3 * j + c]) / ds;
                double Ni = a[i] * (dot3(dd, Dh + 3 * l) - om[i]);
                for (int c = 0; c < 3; c++) Nv[c] += Ni * Dh[3 * i + c];
            }
            memcpy(Fs + 3 * k, F, sizeof F);
            memcpy(Ns + 3 * k, Nv, sizeof Nv);
            memcpy(dXs + 3 * k, dX, sizeof dX);
        }
        for (int32_t k = 0; k < M; k++) {
            double zero[3] = {0, 0, 0};
            const double *Fp = k < nseg ? Fs + 3 * k : zero, *Fm = k > 0 ? Fs + 3 * (k - 1) : zero;
            const double *Np = k < nseg ? Ns + 3 * k : zero, *Nm = k > 0 ? Ns + 3 * (k - 1) : zero;
            const double *Xp = k < nseg ? dXs + 3 * k : zero, *Xm = k > 0 ? dXs + 3 * (k - 1) : zero;
            double tp[3], tm[3], xp[3], xm[3];
            for (int c = 0; c < 3; c++) { xp[c] = Xp[c] / ds; xm[c] = Xm[c] / ds; }
            cross3(xp, Fp, tp);
            cross3(xm, Fm, tm);
            for (int c = 0; c < 3; c++) {
                double fk = -(Fp[c] - Fm[c]) / ds;
                double nk = -(Np[c] - Nm[c]) / ds - 0.5 * (tp[c] + tm[c]);
                g[3 * (k0 + k) + c] = -ds * fk + (fext ? fext[3 * (k0 + k) + c] : 0.0);
                m[3 * (k0 + k) + c] = -ds * nk + (next ? next[3 * (k0 + k) + c] : 0.0);
            }
        }
        free(Fs);
        free(Ns);
        free(dXs);
    }
    if (lj) {
        const int64_t n = off[nfil];
        double *F = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        oracle_lj_forces(nfil, off, X, lj, F);
        for (int64_t i = 0; i < 3 * n; i++) g[i] += F[i];
        free(F);
    }
}

void oracle_rod_forces(int32_t nfil, const int32_t *off, const double *X, const double *D,
                       const double *a, const double *b, const double *om0, double ds,
                       const double *fext, const double *next, double *g, double *m) {
    oracle_rod_forces_ex(nfil, off, X, D, a, b, om0, ds, fext, next, NULL, 0.0, NULL, g, m);
}

/* Elastic energy sum over segments ds (sum_j b_j e_j^2 + sum_i a_i k_i^2)/2 of
 * the strains in Eqs. F_comp_discrete / N_comp_discrete (used by tests to
 * check that relaxation dissipates energy). */
double oracle_rod_energy(int32_t nfil, const int32_t *off, const double *X, const double *D,
                         const double *a, const double *b, const double *om0, double ds) {
    double E = 0.0;
    for (int32_t fi = 0; fi < nfil; fi++) {
        int32_t k0 = off[fi], M = off[fi + 1] - off[fi];
        for (int32_t k = 0; k + 1 < M; k++) {
            const double *Dk = D + 9 * (k0 + k), *Dk1 = D + 9 * (k0 + k + 1);
            double A[9] = {0}, S[9], Dh[9];
            for (int j = 0; j < 3; j++)
                for (int r = 0; r < 3; r++)
                    for (int c = 0; c < 3; c++) A[3 * r + c] += Dk1[3 * j + r] * Dk[3 * j + c];
            oracle_rotsqrt(A, S);
            for (int i = 0; i < 3; i++)
                for (int r = 0; r < 3; r++) {
                    double s = 0.0;
                    for (int c = 0; c < 3; c++) s += S[3 * r + c] * Dk[3 * i + c];
                    Dh[3 * i + r] = s;
                }
            double dX[3];
            for (int c = 0; c < 3; c++) dX[c] = (X[3 * (k0 + k + 1) + c] - X[3 * (k0 + k) + c]) / ds;
            for (int j = 0; j < 3; j++) {
                double e = dot3(dX, Dh + 3 * j) - (j == 2 ? 1.0 : 0.0);
                E += 0.5 * ds * b[j] * e * e;
            }
            for (int i = 0; i < 3; i++) {
                int j = (i + 1) % 3, l = (i + 2) % 3;
                double dd[3];
                for (int c = 0; c < 3; c++) dd[c] = (Dk1[3 * j + c] - Dk[3 * j + c]) / ds;
                double kap = dot3(dd, Dh + 3 * l) - om0[i];
                E += 0.5 * ds * a[i] * kap * kap;
            }
        }
    }
    return E;
}

/* Frame re-orthonormalisation after a step: D3 <- D3/|D3|,
 * D1 <- unit(D1 - (D1.D3) D3), D2 <- D3 x D1. */
void oracle_reorthonormalize(int64_t n, double *D) {
    for (int64_t k = 0; k < n; k++) {
        double *d1 = D + 9 * k, *d2 = D + 9 * k + 3, *d3 = D + 9 * k + 6;
        double l3 = sqrt(dot3(d3, d3));
        for (int c = 0; c < 3; c++) d3[c] /= l3;
        double p = dot3(d1, d3);
        for (int c = 0; c < 3; c++) d1[c] -= p * d3[c];
        double l1 = sqrt(dot3(d1, d1));
        for (int c = 0; c < 3; c++) d1[c] /= l1;
        cross3(d3, d1, d2);
    }
}

/* Rotate every director of every point by Rodrigues(h * omega_k) (Eq. newD). */
static void rotate_frames(int64_t n, const double *W, double h, const double *Din, double *Dout) {
    for (int64_t k = 0; k < n; k++) {
        double v[3] = {h * W[3 * k], h * W[3 * k + 1], h * W[3 * k + 2]};
        for (int i = 0; i < 3; i++) oracle_rodrigues(v, Din + 9 * k + 3 * i, Dout + 9 * k + 3 * i);
    }
}

/* Velocities of a rod state: rod forces plus external loads, then the MRS sum.
 * With include_elastic == 0 only the external loads drive the fluid.  The
 * _ex form adds the swimming waveform at time t (wave may be NULL) to the rod
 * forces and the Lennard-Jones repulsion (lj may be NULL) to the point forces,
 * the latter with or without the elastic forces. */
void oracle_velocities_ex(int32_t nfil, const int32_t *off, const double *X, const double *D,
                          const double *a, const double *b, const double *om0, double ds,
                          const double *fext, const double *next, double eps, double mu,
                          int include_elastic, const double *wave, double t, const double *lj,
                          double *U, double *W) {
    int64_t n = off[nfil];
    double *g = malloc(sizeof(double) * 3 * (size_t)n), *m = malloc(sizeof(double) * 3 * (size_t)n);
    if (include_elastic) {
        oracle_rod_forces_ex(nfil, off, X, D, a, b, om0, ds, fext, next, wave, t, NULL, g, m);
    } else {
        for (int64_t i = 0; i < 3 * n; i++) {
            g[i] = fext ? fext[i] : 0.0;
            m[i] = next ? next[i] : 0.0;
        }
    }
    if (lj) {
        double *F = malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        oracle_lj_forces(nfil, off, X, lj, F);
        for (int64_t i = 0; i < 3 * n; i++) g[i] += F[i];
        free(F);
    }
    oracle_mrs_eval(n, X, g, m, eps, mu, U, W);
    free(g);
    free(m);
}

void oracle_velocities(int32_t nfil, const int32_t *off, const double *X, const double *D,
                       const double *a, const double *b, const double *om0, double ds,
                       const double *fext, const double *next, double eps, double mu,
                       int include_elastic, double *U, double *W) {
    oracle_velocities_ex(nfil, off, X, D, a, b, om0, ds, fext, next, eps, mu, include_elastic, NULL, 0.0,
                         NULL, U, W);
}

/*
 * nsteps explicit steps in place on X, D.
 * integrator 1: forward Euler, X <- X + dt U (Eq. newx),
 *               D^i <- Rodrigues(dt Omega) D^i (Eq. newD).
 * integrator 4: classical RK4 with stage nodes c = (0, 1/2, 1/2, 1) and
 *               weights (1, 2, 2, 1)/6; stage states are
 *               X_s = X + c_s dt U_{s-1}, D_s = Rodrigues(c_s dt Omega_{s-1}) D,
 *               and the step ends with X <- X + dt sum_s w_s U_s,
 *               D <- Rodrigues(dt sum_s w_s Omega_s) D.
 * integrator 2: the second-order Runge-Kutta method the paper's fine
 *               propagator uses (Sec. III.A, n = 2), taken as the midpoint
 *               rule: nodes c = (0, 1/2), weights (0, 1), same stage form.
 * Every step ends with oracle_reorthonormalize.  U, W (may be NULL) receive
 * the velocities of the first stage of the last step.  The _ex form carries
 * the time of the swimming waveform: stage s of a step that starts at time t
 * is evaluated at t + c_s dt, and t advances by dt per step (t in/out, may be
 * NULL for t = 0).
 */
void oracle_step_ex(int32_t nfil, const int32_t *off, double *X, double *D,
                    const double *a, const double *b, const double *om0, double ds,
                    const double *fext, const double *next, double eps, double mu,
                    int integrator, double dt, int32_t nsteps, int include_elastic,
                    const double *wave, double *t, const double *lj, double *Uout, double *Wout) {
    double tnow = t ? *t : 0.0;
    int64_t n = off[nfil];
    size_t v3 = sizeof(double) * 3 * (size_t)n, v9 = sizeof(double) * 9 * (size_t)n;
    double *U = malloc(v3), *W = malloc(v3), *Ua = malloc(v3), *Wa = malloc(v3);
    double *Xs = malloc(v3), *Ds = malloc(v9), *K = malloc(v3);
    for (int32_t step = 0; step < nsteps; step++) {
        if (integrator == 1) {
            oracle_velocities_ex(nfil, off, X, D, a, b, om0, ds, fext, next, eps, mu, include_elastic, wave, tnow,
                                 lj, U, W);
            if (Uout && step == nsteps - 1) memcpy(Uout, U, v3);
            if (Wout && step == nsteps - 1) memcpy(Wout, W, v3);
            for (int64_t i = 0; i < 3 * n; i++) X[i] += dt * U[i];
            rotate_frames(n, W, dt, D, Ds);
            memcpy(D, Ds, v9);
        } else {
            static const double cnode4[4] = {0.0, 0.5, 0.5, 1.0};
            static const double wgt4[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
            static const double cnode2[2] = {0.0, 0.5};
            static const double wgt2[2] = {0.0, 1.0};
            const int nstage = integrator == 2 ? 2 : 4;
            const double *cnode = integrator == 2 ? cnode2 : cnode4;
            const double *wgt = integrator == 2 ? wgt2 : wgt4;
            memset(Ua, 0, v3);
            memset(Wa, 0, v3);
            for (int s = 0; s < nstage; s++) {
                if (s == 0) {
                    memcpy(Xs, X, v3);
                    memcpy(Ds, D, v9);
                } else {
                    for (int64_t i = 0; i < 3 * n; i++) Xs[i] = X[i] + cnode[s] * dt * U[i];
                    rotate_frames(n, W, cnode[s] * dt, D, Ds);
                }
                oracle_velocities_ex(nfil, off, Xs, Ds, a, b, om0, ds, fext, next, eps, mu, include_elastic, wave,
                                     tnow + cnode[s] * dt, lj, U, W);
                if (s == 0 && step == nsteps - 1) {
                    if (Uout) memcpy(Uout, U, v3);
                    if (Wout) memcpy(Wout, W, v3);
                }
                if (nstage == 4 && s > 0) {
                    /* Runge-Kutta-Munthe-Kaas: the stage frame is exp(theta) D with
                     * theta = c_s dt k_{s-1}; the angular velocity there enters as
                     * k_s = dexp^{-1}_theta(Omega) = Omega - theta x Omega / 2 +
                     * theta x (theta x Omega) / 12 (the inverse derivative of the
                     * exponential map on so(3), truncated after the terms a
                     * fourth-order method needs); W holds k_{s-1} on entry to the
                     * stage and k_s after it */
                    for (int64_t k = 0; k < n; k++) {
                        double th[3], t1[3], t2[3];
                        for (int c = 0; c < 3; c++) th[c] = cnode[s] * dt * K[3 * k + c];
                        cross3(th, &W[3 * k], t1);
                        cross3(th, t1, t2);
                        for (int c = 0; c < 3; c++) W[3 * k + c] = W[3 * k + c] - 0.5 * t1[c] + t2[c] / 12.0;
                    }
                }
                if (nstage == 4) memcpy(K, W, v3);
                for (int64_t i = 0; i < 3 * n; i++) {
                    Ua[i] += wgt[s] * U[i];
                    Wa[i] += wgt[s] * W[i];
                }
            }
            for (int64_t i = 0; i < 3 * n; i++) X[i] += dt * Ua[i];
            rotate_frames(n, Wa, dt, D, Ds);
            memcpy(D, Ds, v9);
        }
        oracle_reorthonormalize(n, D);
        tnow += dt;
    }
    if (t) *t = tnow;
    free(U); free(W); free(Ua); free(Wa); free(Xs); free(Ds); free(K);
}

void oracle_step(int32_t nfil, const int32_t *off, double *X, double *D,
                 const double *a, const double *b, const double *om0, double ds,
                 const double *fext, const double *next, double eps, double mu,
                 int integrator, double dt, int32_t nsteps, int include_elastic,
                 double *Uout, double *Wout) {
    oracle_step_ex(nfil, off, X, D, a, b, om0, ds, fext, next, eps, mu, integrator, dt, nsteps, include_elastic,
                   NULL, NULL, NULL, Uout, Wout);
}

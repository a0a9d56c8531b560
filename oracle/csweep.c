/*
 * Plain-C transport sweep for the oracle (test infrastructure only).
 *
 * Paper, Sec. 2.2 ("Transport sweeps"): with upwind DG and cells taken in the
 * upwind order of Omega_j, (D_j + Sigma_t) is block lower triangular, so one
 * block Gauss-Seidel pass solves (D_j + Sigma_t) psi_j = rhs exactly.  This file
 * does that pass cell by cell with the 4x4 cell blocks handed in from Python
 * (oracle/dg.py computes them from the weak form), solving each cell system by
 * Gaussian elimination with partial pivoting.  No vectorisation, no blocking.
 *
 * The transposed pass solves (D_j + Sigma_t)^T mu = rhs: the transposed matrix is
 * block upper triangular in the same order, so cells are taken downwind first and
 * each cell uses the transposed diagonal block and the transposed couplings to the
 * cells that receive from it.
 *
 * Cell (a, b) has index c = b * nx + a and DOFs 4c..4c+3.  Boundary data bnd has
 * shape [4][mb][4] (sides L, R, B, T): bnd[s][i][k] = int_face g eta_k.  In the
 * forward pass a direction gets |Omega.n| bnd on its inflow sides; in the
 * transposed pass the same data is added on its outflow sides (where the
 * derivative of an exit-current functional lives).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Solve M x = r (4x4, row-major) by Gaussian elimination with partial pivoting. */
static void solve4(const double* Min, const double* rin, double* x) {
    double M[4][5];
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) M[i][j] = Min[4 * i + j];
        M[i][4] = rin[i];
    }
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        for (int i = k + 1; i < 4; ++i)
            if (fabs(M[i][k]) > fabs(M[piv][k])) piv = i;
        if (piv != k)
            for (int j = 0; j < 5; ++j) {
                double t = M[k][j]; M[k][j] = M[piv][j]; M[piv][j] = t;
            }
        for (int i = k + 1; i < 4; ++i) {
            double f = M[i][k] / M[k][k];
            for (int j = k; j < 5; ++j) M[i][j] -= f * M[k][j];
        }
    }
    for (int i = 3; i >= 0; --i) {
        double s = M[i][4];
        for (int j = i + 1; j < 4; ++j) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
}

static void one_direction(int nx, int ny, double ox, double oy, const double* A,
                          const double* Bx, const double* By, const double* sigma_t,
                          const double* src, const double* bnd, int mb, double* out,
                          int transpose) {
    /* forward upwind order */
    int a0 = ox >= 0 ? 0 : nx - 1, da = ox >= 0 ? 1 : -1;
    int b0 = oy >= 0 ? 0 : ny - 1, db = oy >= 0 ? 1 : -1;
    if (transpose) { /* downwind first */
        a0 = ox >= 0 ? nx - 1 : 0; da = -da;
        b0 = oy >= 0 ? ny - 1 : 0; db = -db;
    }
    /* sides: 0 L, 1 R, 2 B, 3 T; inflow x side is L when ox > 0 */
    int xin_side = ox > 0 ? 0 : 1, yin_side = oy > 0 ? 2 : 3;
    int xout_side = ox > 0 ? 1 : 0, yout_side = oy > 0 ? 3 : 2;
    double ax = fabs(ox), ay = fabs(oy);
    for (int ib = 0; ib < ny; ++ib) {
        int b = b0 + db * ib;
        for (int ia = 0; ia < nx; ++ia) {
            int a = a0 + da * ia;
            int c = b * nx + a;
            double M[16], r[4], x[4];
            for (int k = 0; k < 4; ++k) r[k] = src[4 * c + k];
            if (!transpose) {
                for (int i = 0; i < 16; ++i) M[i] = A[i];
                for (int k = 0; k < 4; ++k) M[5 * k] += sigma_t[c];
                /* x-upwind neighbour or inflow boundary */
                if (ox != 0.0) {
                    int na = a - (ox > 0 ? 1 : -1);
                    if (na >= 0 && na < nx) {
                        const double* pn = out + 4 * (b * nx + na);
                        for (int k = 0; k < 4; ++k)
                            for (int l = 0; l < 4; ++l) r[k] += Bx[4 * k + l] * pn[l];
                    } else {
                        for (int k = 0; k < 4; ++k) r[k] += ax * bnd[(xin_side * mb + b) * 4 + k];
                    }
                }
                if (oy != 0.0) {
                    int nb = b - (oy > 0 ? 1 : -1);
                    if (nb >= 0 && nb < ny) {
                        const double* pn = out + 4 * (nb * nx + a);
                        for (int k = 0; k < 4; ++k)
                            for (int l = 0; l < 4; ++l) r[k] += By[4 * k + l] * pn[l];
                    } else {
                        for (int k = 0; k < 4; ++k) r[k] += ay * bnd[(yin_side * mb + a) * 4 + k];
                    }
                }
            } else {
                /* transposed diagonal block */
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) M[4 * i + j] = A[4 * j + i];
                for (int k = 0; k < 4; ++k) M[5 * k] += sigma_t[c];
                /* cells that receive from c: x-downwind and y-downwind neighbours */
                if (ox != 0.0) {
                    int na = a + (ox > 0 ? 1 : -1);
                    if (na >= 0 && na < nx) {
                        const double* pn = out + 4 * (b * nx + na);
                        for (int k = 0; k < 4; ++k)
                            for (int l = 0; l < 4; ++l) r[k] += Bx[4 * l + k] * pn[l];
                    } else {
                        for (int k = 0; k < 4; ++k) r[k] += ax * bnd[(xout_side * mb + b) * 4 + k];
                    }
                }
                if (oy != 0.0) {
                    int nb = b + (oy > 0 ? 1 : -1);
                    if (nb >= 0 && nb < ny) {
                        const double* pn = out + 4 * (nb * nx + a);
                        for (int k = 0; k < 4; ++k)
                            for (int l = 0; l < 4; ++l) r[k] += By[4 * l + k] * pn[l];
                    } else {
                        for (int k = 0; k < 4; ++k) r[k] += ay * bnd[(yout_side * mb + a) * 4 + k];
                    }
                }
            }
            solve4(M, r, x);
            for (int k = 0; k < 4; ++k) out[4 * c + k] = x[k];
        }
    }
}

/*
 * Sweep ndir directions.  A, Bx, By: [ndir][16] cell blocks (row = test function).
 * Bx couples to the x-upwind neighbour, By to the y-upwind one.  If psi is not
 * NULL it receives psi_j [ndir][ncell*4]; if phi is not NULL it is overwritten with
 * sum_j w_j psi_j.  Returns 0, or -1 when out of memory.
 */
int oracle_sweep(int nx, int ny, int ndir, const double* Ox, const double* Oy,
                 const double* A, const double* Bx, const double* By,
                 const double* sigma_t, const double* src, const double* bnd, int mb,
                 const double* w, double* psi, double* phi, int transpose, int nthreads) {
    long n4 = 4L * nx * ny;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    double* acc = NULL;
    if (phi) {
        acc = (double*)calloc((size_t)nthreads * n4, sizeof(double));
        if (!acc) return -1;
    }
    double* tmp = NULL;
    if (!psi) {
        tmp = (double*)malloc(sizeof(double) * (size_t)nthreads * n4);
        if (!tmp) { free(acc); return -1; }
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int d = 0; d < ndir; ++d) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* out = psi ? psi + (long)d * n4 : tmp + (long)tid * n4;
        one_direction(nx, ny, Ox[d], Oy[d], A + 16 * d, Bx + 16 * d, By + 16 * d,
                      sigma_t, src, bnd, mb, out, transpose);
        if (acc) {
            double* my = acc + (long)tid * n4;
            for (long i = 0; i < n4; ++i) my[i] += w[d] * out[i];
        }
    }
    free(tmp);
    if (phi) {
        memset(phi, 0, sizeof(double) * n4);
        for (int t = 0; t < nthreads; ++t)
            for (long i = 0; i < n4; ++i) phi[i] += acc[(long)t * n4 + i];
        free(acc);
    }
    return 0;
}

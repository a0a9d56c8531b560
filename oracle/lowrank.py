"""Low-rank SI-DSA of the oracle: Alg. 1 with the low-rank SI of Sec. 3.1-3.4 and Alg. 2.

Steps of one low-rank SI (outer iteration n), in the paper's order (Sec. 3.1):
  1. sweep the p sampled ordinates, eq. (sampled-sweep);
  2. MGS2-A (Alg. 2): append the snapshots to the spatial basis X, R gets a column
     (c, alpha) per snapshot; snapshots of one batch are processed one after the
     other (Sec. 3.4);
  3. incremental update of the projected operators X^T Sigma_t X, X^T D_x^{+-} X,
     X^T D_y^{+-} X and the projected right-hand sides (Sec. 3.4, bordering);
  4. q random previously unsampled candidates, Galerkin projection
     eq. (galerkin-projection), residuals, greedy choice of the p largest (Sec. 3.2);
  5. stopping test (Sec. 3.3): residual check eq. (residual-chk), then the full
     projection phi^{n,k} = X (C w) and the test eq. (phi-diff);
  6. after the inner loop, the truncated SVD C = U S V^T and X^{n} = X U (Sec. 3.3).

Readings (also implemented by the GPU library):
  * X is empty at the start of every outer iteration and p initial angles are
    drawn at random (r_k = p k, Sec. 3.2 "Initial sampling");
  * "angles" in the sampling are the distinct (Omega_x, Omega_y) of the ordinate set:
    in 2D X-Y geometry D_j depends on Omega_j only through (Omega_x, Omega_y)
    (eq. (upwind-operator)), so ordinates with equal (Omega_x, Omega_y) (the Omega_z
    twins of the full-sphere CL rule) share eq. (SI), its sweep and its Galerkin
    projection; one sweep samples the whole class and candidates are drawn among
    unsampled classes.  (Sampling a twin separately adds nothing to X, and two
    consecutive stop checks with an unchanged X pass the phi-difference test
    spuriously);
  * the residual source Sigma_s phi^{(k)} is read as Sigma_s phi^{n-1} (the source of
    eq. (sampled-sweep)); eps_res and eps_diff are absolute thresholds on the
    coefficient 2-norm;
  * random draws: a caller-supplied stream of uint64 values u; a draw of k items from
    the ascending list of n unsampled class indices is a partial Fisher-Yates shuffle with
    swap index i + floor(u (n - i) / 2^64); candidates are all unsampled ordinates
    when fewer than q remain;
  * classes are numbered in the order of their smallest ordinate index; greedy order:
    residual norm descending, class index ascending on ties, where norms are compared
    after rounding their binary mantissa to 30 bits (angles related by a symmetry of
    the medium have residuals that are equal in exact arithmetic and differ only by
    rounding; the paper does not say how ties are broken);
  * a forced (replayed) sample sequence is given per outer iteration; if the inner
    loop needs more groups than given, the greedy choice takes over;
  * the next samples are the top p of the current candidates, also after a failed
    phi-difference test; the inner loop also ends when every class is sampled;
  * MGS2-A breakdown (not specified by the paper): if alpha <= tol_break * ||psi||,
    the snapshot is not appended and the sampled class keeps the coefficient c;
  * truncation rank r' = smallest l with sum_{i>l} s_i <= eps_svd sum_i s_i;
  * basis-update variants of Sec. 4.2 (the paper gives no listing for them):
    - "mgs_qr": one block projection (the Delta c = X^T psi of Alg. 2), normalisation and
      the orthogonality test against X(:,1); when the test fails, a full QR of the matrix
      of all snapshots of the outer iteration replaces the basis;
    - "full_qr": after every batch of sampled snapshots, a full QR of the matrix of all
      snapshots of the outer iteration replaces the basis;
    a full QR is the Householder QR of the snapshot matrix (LAPACK) with the signs fixed
    so that diag(R) > 0; the sampled classes take the columns of R as coefficients, and
    the projected operators and right-hand sides are recomputed from the new basis (the
    incremental bordering needs the nested basis that a full QR does not keep);
  * DEIM sampling (the alternative of the Remark in Sec. 3.2; the paper gives no
    listing): the stopping test is unchanged (q random candidates and their residuals);
    the next samples come from C^{(n,k)} = [c_1 .. c_{N_Omega}] (R columns for sampled
    angles, Galerkin coefficients for all others), its thin SVD C = U S V^T and the DEIM
    indices (Chaturantabut-Sorensen greedy interpolation points) of the leading r'
    columns of V, r' by the truncation rule with eps_svd; the rows of V are taken per
    class (twins have equal columns in C, hence equal rows in V).  The next p samples
    are the first p DEIM indices that are unsampled classes; when there are fewer, the
    candidates in greedy residual order fill the rest.  A DEIM maximum is taken over the
    unpicked rows with the 30-bit key of the greedy order, the lower class index on ties,
    and the point selection stops once p unsampled classes are picked.
"""
import math

import numpy as np
import scipy.linalg as sla

from . import dg, sweep

MASK64 = (1 << 64) - 1


class RandomStream:
    """Consumes a caller-given array of uint64 values in order."""

    def __init__(self, values):
        self.v = np.asarray(values, dtype=np.uint64)
        self.i = 0

    def next(self):
        if self.i >= self.v.size:
            raise RuntimeError("random stream exhausted")
        u = int(self.v[self.i])
        self.i += 1
        return u


def order_key(res):
    """Comparison key of a residual norm: (binary exponent, mantissa rounded to 30 bits)."""
    if res <= 0.0:
        return (-100000, 0)
    m, e = math.frexp(res)              # res = m 2^e, 0.5 <= m < 1
    q = int(math.floor(m * (1 << 30) + 0.5))
    if q == (1 << 30):
        return (e + 1, 1 << 29)
    return (e, q)


def draw(stream, pool, k):
    """Draw k distinct items from the ascending list `pool` (partial Fisher-Yates)."""
    arr = sorted(int(x) for x in pool)
    n = len(arr)
    k = min(k, n)
    for i in range(k):
        u = stream.next()
        j = i + ((u * (n - i)) >> 64)
        arr[i], arr[j] = arr[j], arr[i]
    return arr[:k]


def truncation_rank(s, eps_svd):
    """Smallest l with sum_{i>l} s_i <= eps_svd * sum_i s_i (l1 tail, Sec. 4 setting)."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0:
        return 0
    total = s.sum()
    if total == 0.0:
        return 0
    for l in range(s.size + 1):
        if s[l:].sum() <= eps_svd * total:
            return l
    return s.size


def deim_indices(V, stop=None):
    """DEIM interpolation indices of the columns of V (Chaturantabut-Sorensen): index l
    maximises |rho| with rho = v_l - V_l (P^T V_l)^{-1} P^T v_l, the error of interpolating
    column l at the indices P picked so far from the previous columns V_l.  Rows already
    picked are skipped; `stop(idx)` ends the selection early."""
    V = np.asarray(V, dtype=np.float64)
    K, m = V.shape
    idx = []
    zero = order_key(0.0)
    for l in range(m):
        v = V[:, l]
        if idx:
            coef = np.linalg.solve(V[idx, :l], v[idx])
            rho = v - V[:, :l] @ coef
        else:
            rho = v.copy()
        best, bi = None, -1
        for i in range(K):
            if i in idx:
                continue
            key = order_key(abs(float(rho[i])))
            if best is None or key > best:   # first maximum: lower index on ties
                best, bi = key, i
        if best is None or best == zero:
            break
        idx.append(bi)
        if stop is not None and stop(idx):
            break
    return idx


def direction_classes(dirs, tol=1e-12):
    """Group ordinates with equal (Omega_x, Omega_y); classes ordered by smallest member.

    Returns (cls [N] class id of each ordinate, reps [K] smallest ordinate of each class).
    """
    n = len(dirs)
    cls = -np.ones(n, dtype=np.int64)
    reps = []
    for j in range(n):
        if cls[j] >= 0:
            continue
        cls[j] = len(reps)
        for i in range(j + 1, n):
            if cls[i] < 0 and abs(dirs[i, 0] - dirs[j, 0]) <= tol and abs(dirs[i, 1] - dirs[j, 1]) <= tol:
                cls[i] = len(reps)
        reps.append(j)
    return cls, np.array(reps, dtype=np.int64)


def _project_out(X, v):
    """One classical Gram-Schmidt pass: (v - X X^T v, X^T v)."""
    dc = X.T @ v
    return v - X @ dc, dc


class LowRankSI:
    """One low-rank SI solve (Sec. 3.1) for a fixed source Sigma_s phi^{n-1} + G."""

    def __init__(self, prob, ops, p, q, eps_res, eps_diff, eps_mgs=1e-10, m_max=4,
                 tol_break=1e-12, nthreads=0, basis_update="mgs2a", sampling="greedy",
                 eps_svd=1e-8):
        self.prob, self.ops = prob, ops
        self.p, self.q = p, q
        self.eps_res, self.eps_diff = eps_res, eps_diff
        self.eps_mgs, self.m_max, self.tol_break = eps_mgs, m_max, tol_break
        self.nthreads = nthreads
        assert basis_update in ("mgs2a", "mgs_qr", "full_qr"), basis_update
        self.basis_update = basis_update
        assert sampling in ("greedy", "deim"), sampling
        self.sampling, self.eps_svd = sampling, eps_svd
        self.extra = None   # [N_Omega][ndof] angular source added to eq. (SI) (time steps)

    # ---------------- Alg. 2 (MGS2-A) ----------------
    def mgs2a_append(self, psi):
        """Alg. 2 for one snapshot: block Gram-Schmidt against the current basis X,
        repeated where the orthogonality test against the first basis vector fails, then
        append the normalised remainder.

        The remainder v and the coefficient vector satisfy psi = X coef + v at every
        stage.  Two projection passes always run; then, while the normalised remainder
        u = v/alpha still has a component above eps_mgs along X(:,1), the un-normalised
        alpha u is projected again (at most m_max more times).  Returns the R column
        (coef, alpha) and whether the snapshot was appended; a remainder of relative size
        tol_break or less is not appended (breakdown: psi already lies in span(X)).
        """
        X = self.X
        r = X.shape[1]
        coef = np.zeros(r)
        v = psi.copy()
        for _ in range(2):
            v, dc = _project_out(X, v)
            coef = coef + dc
        alpha = float(np.linalg.norm(v))
        if alpha <= self.tol_break * float(np.linalg.norm(psi)):
            self.breakdowns += 1
            return coef, False
        u = v / alpha

        def leaks(u):
            return r > 0 and abs(float(X[:, 0] @ u)) > self.eps_mgs

        extra = 0
        while extra < self.m_max and leaks(u):
            v, dc = _project_out(X, alpha * u)
            coef = coef + dc
            alpha = float(np.linalg.norm(v))
            u = v / alpha
            extra += 1
        if leaks(u):
            self.mgs_failures += 1
        self.X = np.concatenate([X, u[:, None]], axis=1)
        return np.append(coef, alpha), True

    # ---------------- basis-update variants of Sec. 4.2 ----------------
    def full_qr(self):
        """Replace X by the Q of a full QR of all snapshots of this outer iteration (in
        sampling order); the sampled classes get the columns of R as coefficients and the
        projected operators are recomputed.  A snapshot whose diagonal entry of R is at
        most tol_break times its norm is already in the span of the earlier ones: it adds
        no column and keeps its projection as coefficients (as a breakdown in Alg. 2)."""
        self.full_qrs += 1
        S = np.stack([psi for _, psi in self.snaps], axis=1)
        Rd = np.abs(np.diag(np.linalg.qr(S, mode="r")))
        keep = [i for i, (_, psi) in enumerate(self.snaps)
                if Rd[i] > self.tol_break * float(np.linalg.norm(psi))]
        Q, R = np.linalg.qr(S[:, keep])
        Q = Q * np.where(np.diag(R) < 0.0, -1.0, 1.0)[None, :]
        self.X = Q
        for c, psi in self.snaps:
            self.coef[c] = Q.T @ psi
        self._project_fresh()

    def _project_fresh(self):
        """Projected operators and right-hand sides of the current basis from scratch."""
        X, o = self.X, self.ops
        self.T = X.T @ (o["Sig_t"] @ X)
        self.Dxm = X.T @ (o["Dxm"] @ X); self.Dxp = X.T @ (o["Dxp"] @ X)
        self.Dym = X.T @ (o["Dym"] @ X); self.Dyp = X.T @ (o["Dyp"] @ X)
        self.b_src = X.T @ self.src
        self.b_side = (X.T @ o["gside"].T).T

    def mgs_qr_append(self, c, psi):
        """One block projection of the snapshot, then the orthogonality test against
        X(:,1); on failure a full QR of all snapshots replaces the basis.  Returns True
        when the basis was replaced (the projected operators are then already fresh)."""
        self.snaps.append((c, psi.copy()))
        X = self.X
        r = X.shape[1]
        dc = X.T @ psi
        v = psi - X @ dc
        alpha = float(np.linalg.norm(v))
        if alpha <= self.tol_break * float(np.linalg.norm(psi)):
            self.breakdowns += 1
            self.coef[c] = dc
            return False
        u = v / alpha
        if r > 0 and abs(float(X[:, 0] @ u)) > self.eps_mgs:
            self.full_qr()
            return True
        self.X = np.concatenate([X, u[:, None]], axis=1)
        self.coef[c] = np.append(dc, alpha)
        return False

    # ---------------- incremental bordering (Sec. 3.4) ----------------
    def border(self, P):
        """Grow the projected operators and right-hand sides by the new columns P."""
        if P.shape[1] == 0:
            return
        X = self.X                      # already contains P as its last columns
        r_old = X.shape[1] - P.shape[1]
        Xo = X[:, :r_old]
        o = self.ops

        def grow(M, Aop):
            AP = Aop @ P                # new column block  X^T (A P)
            ATP = Aop.T @ P             # new row block     P^T A X_old = (X_old^T A^T P)^T
            col = X.T @ AP
            row = (Xo.T @ ATP).T
            out = np.zeros((X.shape[1], X.shape[1]))
            out[:r_old, :r_old] = M
            out[:, r_old:] = col
            out[r_old:, :r_old] = row
            return out

        self.T = grow(self.T, o["Sig_t"])
        self.Dxm = grow(self.Dxm, o["Dxm"]); self.Dxp = grow(self.Dxp, o["Dxp"])
        self.Dym = grow(self.Dym, o["Dym"]); self.Dyp = grow(self.Dyp, o["Dyp"])
        self.b_src = np.concatenate([self.b_src, P.T @ self.src])
        self.b_side = np.concatenate([self.b_side, (P.T @ o["gside"].T).T], axis=1)

    # ---------------- Galerkin projection, eq. (galerkin-projection) ----------------
    def reduced_system(self, j):
        """X^T (D_j + Sigma_t) X and X^T (Sigma_s phi^{n-1} + G~_j) for ordinate j."""
        ox, oy = self.prob.dirs[j, 0], self.prob.dirs[j, 1]
        A = self.T.copy()
        A += ox * (self.Dxm if ox >= 0 else self.Dxp)
        A += oy * (self.Dym if oy >= 0 else self.Dyp)
        b = self.b_src.copy()
        if self.extra is not None:
            b += self.X.T @ self.extra[j]
        if ox > 0: b += ox * self.b_side[0]
        elif ox < 0: b += -ox * self.b_side[1]
        if oy > 0: b += oy * self.b_side[2]
        elif oy < 0: b += -oy * self.b_side[3]
        return A, b

    def galerkin(self, j):
        A, b = self.reduced_system(j)
        return sla.solve(A, b)

    def residual_norm(self, j, c):
        """||Sigma_s phi^{n-1} + G~_j - (D_j + Sigma_t) X c||_2 (Sec. 3.2)."""
        o = self.ops
        ox, oy = self.prob.dirs[j, 0], self.prob.dirs[j, 1]
        v = self.X @ c
        Dv = ox * ((o["Dxm"] if ox >= 0 else o["Dxp"]) @ v) + oy * ((o["Dym"] if oy >= 0 else o["Dyp"]) @ v)
        res = self.src + self.prob.g_bc(j) - Dv - o["Sig_t"] @ v
        if self.extra is not None:
            res = res + self.extra[j]
        return float(np.linalg.norm(res))

    def class_coefficients(self):
        """Coefficients of every class: R columns if sampled, Galerkin otherwise."""
        r = self.X.shape[1]
        K = len(self.reps)
        Cc = np.zeros((r, K))
        for c in range(K):
            if c in self.coef:
                cc = self.coef[c]
                Cc[:cc.size, c] = cc
            else:
                Cc[:, c] = self.galerkin(self.reps[c])
        return Cc

    def deim_samples(self, order):
        """The next p samples by DEIM on the angular basis (Remark in Sec. 3.2)."""
        Cc = self.class_coefficients()
        C = Cc[:, self.cls]                          # r x N_Omega
        _, s, Vt = np.linalg.svd(C, full_matrices=False)
        m = truncation_rank(s, self.eps_svd)
        Vc = Vt[:m].T[self.reps]                     # one row per class
        uns = lambda idx: sum(1 for c in idx if c not in self.coef)
        picked = [c for c in deim_indices(Vc, stop=lambda idx: uns(idx) >= self.p)
                  if c not in self.coef]
        for c in order:
            if len(picked) >= self.p:
                break
            if c not in picked:
                picked.append(c)
        return picked[:self.p]

    # ---------------- the inner loop (Sec. 3.1-3.3) ----------------
    def run(self, src, phi_prev, stream, replay=None):
        """Low-rank SI for the source `src`.  `replay` forces the sampled classes per
        inner iteration (a list of lists of class ids)."""
        prob = self.prob
        n = prob.mesh.ndof
        self.cls, self.reps = direction_classes(prob.dirs)
        K = len(self.reps)
        wc = np.zeros(K)
        np.add.at(wc, self.cls, prob.w)
        self.src = src
        self.X = np.zeros((n, 0))
        self.T = np.zeros((0, 0)); self.Dxm = self.T.copy(); self.Dxp = self.T.copy()
        self.Dym = self.T.copy(); self.Dyp = self.T.copy()
        self.b_src = np.zeros(0); self.b_side = np.zeros((4, 0))
        self.coef = {}
        self.snaps = []                 # (class, snapshot) of this outer iteration
        self.mgs_failures = 0
        self.breakdowns = 0
        self.full_qrs = 0
        self.n_swept = 0
        log = []
        phi_old = phi_prev.copy()
        k = 0
        samples = list(replay[0]) if replay else draw(stream, range(K), self.p)
        while True:
            k += 1
            # 1. sweeps of the sampled angles, eq. (sampled-sweep)
            if self.extra is None:
                psi, _ = sweep.sweep(prob.mesh, prob.dirs, self.reps[samples], prob.sigma_t, src,
                                     prob.bnd, want_psi=True, nthreads=self.nthreads)
            else:   # the angular source differs per class: one sweep each
                psi = np.concatenate([
                    sweep.sweep(prob.mesh, prob.dirs, self.reps[[c]], prob.sigma_t,
                                src + self.extra[self.reps[c]], prob.bnd, want_psi=True,
                                nthreads=self.nthreads)[0] for c in samples])
            self.n_swept += len(samples)
            # 2. basis update: MGS2-A (Alg. 2), one snapshot after the other, or a variant
            # of Sec. 4.2;  3. bordering with the appended columns (MGS2-A), or the
            # operators recomputed after a full QR
            r_before = self.X.shape[1]
            if self.basis_update != "mgs_qr":
                self.snaps.extend((c, psi[i].copy()) for i, c in enumerate(samples))
            if self.basis_update == "mgs2a":
                for i, c in enumerate(samples):
                    col, _ = self.mgs2a_append(psi[i])
                    self.coef[c] = col
                self.border(self.X[:, r_before:])
            elif self.basis_update == "full_qr":
                self.full_qr()
            else:
                fresh = False
                for i, c in enumerate(samples):
                    if self.mgs_qr_append(c, psi[i]):
                        fresh = True
                if fresh:
                    self._project_fresh()
                else:
                    self.border(self.X[:, r_before:])
            entry = dict(k=k, samples=list(samples), rank=self.X.shape[1])
            unsampled = [c for c in range(K) if c not in self.coef]
            if not unsampled:
                Cc = self.class_coefficients()
                phi = self.X @ (Cc @ wc)
                entry.update(stop="all_sampled")
                log.append(entry)
                break
            # 4. candidates, Galerkin, residuals
            cand = draw(stream, unsampled, self.q)
            res = {c: self.residual_norm(self.reps[c], self.galerkin(self.reps[c])) for c in cand}
            entry.update(candidates=list(cand), residuals=[res[c] for c in cand])
            order = sorted(cand, key=lambda c: (tuple(-x for x in order_key(res[c])), c))
            # 5. stopping test, Sec. 3.3
            stop = False
            if max(res.values()) < self.eps_res:
                Cc = self.class_coefficients()
                phi = self.X @ (Cc @ wc)
                dphi = float(np.linalg.norm(phi - phi_old))
                entry.update(phi_diff=dphi)
                if dphi <= self.eps_diff:
                    stop = True
                else:
                    phi_old = phi
            log.append(entry)
            if stop:
                break
            if replay is not None and k < len(replay):
                samples = list(replay[k])
            elif self.sampling == "deim":
                samples = self.deim_samples(order)
            else:
                samples = order[:self.p]
        self.C = Cc[:, self.cls]            # r x N_Omega, every ordinate takes its class column
        self.phi = phi
        self.log = log
        return phi

    def truncate(self, eps_svd):
        """Truncated SVD of C and X^{n} = X U (Sec. 3.3, construction after convergence)."""
        U, s, Vt = np.linalg.svd(self.C, full_matrices=False)
        rp = truncation_rank(s, eps_svd)
        return self.X @ U[:, :rp], s[:rp], Vt[:rp].T, s


def operators(prob):
    """The sparse operators the low-rank SI needs (Appendix B)."""
    Dxm, Dxp, Dym, Dyp = dg.directional_operators(prob.mesh)
    mesh = prob.mesh
    gside = np.zeros((4, mesh.ndof))
    # unit boundary vectors of the four sides (per unit |Omega . n|)
    for s, (ox, oy) in enumerate(((1.0, 0.0), (-1.0, 0.0), (0.0, 1.0), (0.0, -1.0))):
        gside[s] = dg.boundary_vector(mesh, prob.bnd, ox, oy)
    return dict(Dxm=Dxm.tocsr(), Dxp=Dxp.tocsr(), Dym=Dym.tocsr(), Dyp=Dyp.tocsr(),
                Sig_t=dg.cell_sigma_diag(mesh, prob.sigma_t).tocsr(), gside=gside)


def lr_si_dsa(prob, eps_si, p, q, eps_res, eps_diff, eps_svd, rand, eps_mgs=1e-10, m_max=4,
              max_outer=100, phi0=None, use_dsa=True, replay=None, tol_break=1e-12,
              nthreads=0, keep_factors=True, basis_update="mgs2a", sampling="greedy",
              extra=None):
    """Alg. 1.  `rand` is the uint64 stream; `replay` optionally forces samples per outer;
    `extra` [N_Omega][ndof] is an angular source added to the right-hand side of every
    ordinate's transport equation (the psi^m / dt of a backward Euler step)."""
    ops = operators(prob)
    stream = RandomStream(rand)
    phi_prev = np.zeros(prob.mesh.ndof) if phi0 is None else np.asarray(phi0, dtype=np.float64).copy()
    hist, logs, ranks, sampled, phis = [], [], [], [], []
    lr = LowRankSI(prob, ops, p, q, eps_res, eps_diff, eps_mgs, m_max, tol_break, nthreads,
                   basis_update, sampling, eps_svd)
    lr.extra = None if extra is None else np.asarray(extra, dtype=np.float64)
    mgs_fail = breakdowns = full_qrs = 0
    out = None
    phi_star = phi_prev
    for n in range(1, max_outer + 1):
        src = prob.sig_s4 * phi_prev + prob.G
        rep = None if replay is None or n - 1 >= len(replay) else replay[n - 1]
        phi_star = lr.run(src, phi_prev, stream, rep)
        phis.append(phi_star)
        mgs_fail += lr.mgs_failures
        breakdowns += lr.breakdowns
        full_qrs += lr.full_qrs
        Xn, S, V, s_all = lr.truncate(eps_svd)
        ranks.append(S.size)
        sampled.append(lr.n_swept)
        logs.append(lr.log)
        d = float(np.max(np.abs(phi_star - phi_prev)))
        hist.append(d)
        if d <= eps_si:
            out = dict(phi=phi_star, iters=n, converged=True)
            break
        phi_prev = phi_star + prob.dsa().correction(phi_star, phi_prev) if use_dsa else phi_star
    if out is None:
        out = dict(phi=phi_star, iters=max_outer, converged=False)
    out.update(history=hist, logs=logs, ranks=ranks, n_sampled=sampled, phis=phis, mgs_failures=mgs_fail,
               breakdowns=breakdowns, full_qrs=full_qrs, rand_used=stream.i)
    if keep_factors:
        out.update(X=Xn, S=S, V=V, singular_values=s_all, C=lr.C, Xfull=lr.X)
    return out

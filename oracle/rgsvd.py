"""FP64 CPU oracle of the randomized GSVD (test infrastructure only).

Plain, slow, obviously-correct NumPy/LAPACK code that follows the paper step
by step; it shares no code with the HIP path.  Only tests, the smoke check and
the benchmark's CPU-baseline leg may import it.

Paper map (arXiv 2404.09459):
  * GMP and reduced GSVD G1 = U S1 R, G2 = V S2 R, alpha^2 + beta^2 = 1,
    alpha descending ............................. Sec. 1, eqs. (gsvd1), (ab)
  * comparative quantities rho, theta, P, D ...... Sec. 1, eqs.
    (antisymmetric-angular-distance), (generalized-fraction),
    (generalized-shannon-entropy)
  * randomized basis extraction .................. Sec. 2, Algorithm 1
  * fixed sketch of k+p columns .................. Sec. 3, Theorem "projector"
  * compressed pair, stacked reduced QR, SVD of L1,
    zero append, beta from alpha ................. Sec. 2, eq. (gsvd-reduced), Algorithm 2
  * GSVD recovery U, V, R ........................ Sec. 2, text after Algorithm 2

Readings taken where the paper is silent or does not apply as written:
  * Power (subspace) iterations W = orth(G^T Q), Q = orth(G W) are not in the
    paper; they follow Halko-Martinsson-Tropp's subspace iteration (the
    paper's ref. [hmt11]).  q counts (G^T, G) pairs.
  * Orthonormalisation is the reduced QR of the paper with the sign of each
    column fixed so that diag(T) > 0 (the QR is then unique for full-rank Y,
    as used in the proof of Lemma c2).
  * Truncation (the main reading): the stacked reduced QR of Algorithm 2 needs
    l1 + l2 >= n.  When l1 + l2 < n its literal result has orthonormal rows
    and every alpha equals 1.  The oracle then keeps the dominant rank-t
    joint row space of the stacked pair (thin SVD B = U_B S_B W_B^T,
    L = U_B[:, :t], R~ = S_t W_t^T) and applies Algorithm 2's CS step to
    L = [L1; L2].  For t = n <= l1 + l2 this is the paper's Algorithm 2 up to
    a right orthogonal factor of R~.
  * beta is taken as the column norms of L2 Y (L1 = X1 C Y^T), which keeps
    full absolute accuracy when alpha ~ 1; the paper's rule
    beta = sqrt(1 - alpha^2) is returned alongside as a cross-check.
  * theta uses atan2(alpha, beta) - pi/4, which equals the paper's arctan of
    the ratio and yields pi/4 when beta = 0 (rho = infinity).
  * Entropy sums and log t run over the t returned pairs, 0 log 0 = 0, and
    D = 0 for t = 1.
  * Signs: each row of R has its largest-magnitude entry positive; U and V
    columns follow.
"""
import numpy as np

from .philox import gaussian_matrix, STREAM_G1, STREAM_G2

BETA_ZERO = 1e-14


# ----------------------------------------------------------------- basics ---
def qr_pos(Y):
    """Reduced Householder QR (LAPACK) with diag(T) made positive."""
    Q, T = np.linalg.qr(Y, mode="reduced")
    s = np.sign(np.diag(T))
    s[s == 0] = 1.0
    return Q * s[None, :], T * s[:, None]


# ----------------------------------------------------- basis extraction ---
def basis_fixed(G, l, q, seed, stream):
    """Randomized range basis with a fixed sketch of l = k + p columns.

    Sketch Y = G Omega with Omega n x l Gaussian (Theorem "projector"), reduced
    QR (Algorithm 1's QR step), then q subspace iterations.
    Returns (Q, info) with Q of shape m x l.
    """
    n = G.shape[1]
    Om = gaussian_matrix(seed, stream, n, 0, l)
    Q, _ = qr_pos(G @ Om)
    for _ in range(q):
        W, _ = qr_pos(G.T @ Q)
        Q, _ = qr_pos(G @ W)
    return Q


BLOCK_DROP = 1e-5


def _orth_block(Y, Q):
    """Orthonormal columns for the block Y against the basis Q so far: the
    reduced QR of (I - QQ^T) Y with a positive diagonal, taken column by column
    (Gram-Schmidt against Q and the block's earlier columns, applied twice).
    A column whose projected norm is below BLOCK_DROP times its own norm lies
    numerically in the span already formed; it is returned as a zero column so
    that the nonzero columns of [Q, P] stay orthonormal (normalising the
    rounding residue instead would give a direction that is not orthogonal to
    Q and count energy twice in the residual)."""
    P = np.zeros_like(Y)
    for j in range(Y.shape[1]):
        y = Y[:, j]
        v = y.copy()
        for _ in range(2):
            v = v - Q @ (Q.T @ v)
            v = v - P[:, :j] @ (P[:, :j].T @ v)
        nv = np.linalg.norm(v)
        if nv > BLOCK_DROP * np.linalg.norm(y) and nv > 0:
            P[:, j] = v / nv
    return P


def basis_adaptive(G, eps, b, seed, stream, lmax=None, rel=False):
    """Algorithm 1: blocks of b Gaussian columns until ||(I - QQ^T)G||_F < eps.

    Each block: Y_i = (I - QQ^T) G Omega_i (the projection applied twice),
    reduced QR Y_i = P_i T_i, Q = [Q, P_i]; columns of a block that are
    numerically inside span(Q) become zero columns (see _orth_block).  The residual is kept in the
    cumulative form of Sec. 2: ||G||_F^2 - sum_i ||P_i^T G||_F^2, floored at
    zero.  Blocks use consecutive global columns of one Omega stream.
    The loop runs over ceil(min(m, n)/b) blocks with a short last block.
    With rel=True the test is against eps * ||G||_F.
    Returns (Q, residual_history).
    """
    m, n = G.shape
    lcap = min(m, n) if lmax is None else min(lmax, m, n)
    normG2 = float(np.sum(G * G))
    thresh = eps * np.sqrt(normG2) if rel else eps
    Q = np.zeros((m, 0))
    energy = 0.0
    hist = []
    col = 0
    while col < lcap:
        bb = min(b, lcap - col)
        Y = G @ gaussian_matrix(seed, stream, n, col, bb)
        P = _orth_block(Y, Q)
        Q = np.hstack([Q, P])
        Bt = P.T @ G
        energy += float(np.sum(Bt * Bt))
        res = np.sqrt(max(0.0, normG2 - energy))
        hist.append(res)
        col += bb
        if res < thresh:
            break
    return Q, hist


# ------------------------------------------------------- small GSVD step ---
def cs_step(B1, B2, t):
    """Compressed-pair GSVD (Algorithm 2 with the truncation reading).

    B1 (l1 x n), B2 (l2 x n).  Returns dict with alpha, beta, X1 (l1 x t),
    X2 (l2 x t), R (t x n), sigma_B (all singular values of the stack).
    """
    l1 = B1.shape[0]
    n = B1.shape[1]
    B = np.vstack([B1, B2])
    UB, sB, WBt = np.linalg.svd(B, full_matrices=False)
    L = UB[:, :t]
    Rt = sB[:t, None] * WBt[:t, :]
    L1, L2 = L[:l1], L[l1:]
    # SVD of L1; right factor complete (t x t) so that alpha is zero-appended
    # when l1 < t (Algorithm 2, "append zeros").
    X1f, c, Yt = np.linalg.svd(L1, full_matrices=True)
    alpha = np.zeros(t)
    alpha[:len(c)] = c
    Y = Yt.T
    X1 = np.zeros((l1, t))
    kk = min(l1, t)
    X1[:, :kk] = X1f[:, :kk]
    L2Y = L2 @ Y
    beta = np.sqrt(np.sum(L2Y * L2Y, axis=0))
    X2 = np.zeros_like(L2Y)
    ok = beta > BETA_ZERO
    X2[:, ok] = L2Y[:, ok] / beta[ok]
    R = Y.T @ Rt
    # sign convention: the largest-magnitude entry of each row of R positive
    idx = np.argmax(np.abs(R), axis=1)
    s = np.sign(R[np.arange(t), idx])
    s[s == 0] = 1.0
    return dict(alpha=alpha, beta=beta, X1=X1 * s, X2=X2 * s,
                R=R * s[:, None], sigma_B=sB,
                beta_paper=np.sqrt(np.maximum(0.0, 1.0 - alpha * alpha)))


def quantities(alpha, beta):
    """theta, rho, P1, P2, D1, D2 of Sec. 1 over the t given pairs."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    t = alpha.shape[0]
    theta = np.arctan2(alpha, beta) - np.pi / 4
    with np.errstate(divide="ignore"):
        rho = np.where(beta > 0, alpha / np.where(beta > 0, beta, 1.0), np.inf)
    a2, b2 = alpha * alpha, beta * beta
    P1 = a2 / np.sum(a2)
    P2 = b2 / np.sum(b2)

    def ent(P):
        if t <= 1:
            return 0.0
        nz = P > 0
        return float(-np.sum(P[nz] * np.log(P[nz])) / np.log(t))

    return dict(theta=theta, rho=rho, P1=P1, P2=P2, D1=ent(P1), D2=ent(P2))


# ------------------------------------------------------------ full method ---
def rgsvd(G1, G2, k, oversample, q, seed, t=None, l1=None, l2=None):
    """Randomized GSVD of the pair (fixed sketch size), FP64.

    l_i = k + oversample unless given; t = k unless given.
    Returns dict: alpha, beta, U (m x t), V (p x t), R (t x n), theta, rho,
    P1, P2, D1, D2, Q1, Q2, B1, B2, sigma_B, beta_paper.
    """
    G1 = np.asarray(G1, dtype=np.float64)
    G2 = np.asarray(G2, dtype=np.float64)
    l1 = k + oversample if l1 is None else l1
    l2 = k + oversample if l2 is None else l2
    t = k if t is None else t
    Q1 = basis_fixed(G1, l1, q, seed, STREAM_G1)
    Q2 = basis_fixed(G2, l2, q, seed, STREAM_G2)
    return finish(G1, G2, Q1, Q2, t)


def finish(G1, G2, Q1, Q2, t):
    """Projection B_i = Q_i^T G_i, compressed GSVD, recovery and quantities."""
    B1 = Q1.T @ G1
    B2 = Q2.T @ G2
    cs = cs_step(B1, B2, t)
    out = dict(cs)
    out.update(Q1=Q1, Q2=Q2, B1=B1, B2=B2,
               U=Q1 @ cs["X1"], V=Q2 @ cs["X2"])
    out.update(quantities(cs["alpha"], cs["beta"]))
    return out


def full_gsvd(G1, G2):
    """Deterministic GSVD of a GMP: Algorithm 2 with Q1 = I, Q2 = I.

    Stacked reduced QR [G1; G2] = [L1; L2] R~ (needs m + p >= n), SVD of L1,
    zero-append, beta from L2.  Used on tiny inputs.
    """
    G1 = np.asarray(G1, dtype=np.float64)
    G2 = np.asarray(G2, dtype=np.float64)
    m, n = G1.shape
    L, Rt = np.linalg.qr(np.vstack([G1, G2]), mode="reduced")
    L1, L2 = L[:m], L[m:]
    X1f, c, Yt = np.linalg.svd(L1, full_matrices=True)
    alpha = np.zeros(n)
    alpha[:len(c)] = c
    Y = Yt.T
    L2Y = L2 @ Y
    beta = np.sqrt(np.sum(L2Y * L2Y, axis=0))
    X1 = np.zeros((m, n))
    kk = min(m, n)
    X1[:, :kk] = X1f[:, :kk]
    X2 = np.zeros_like(L2Y)
    ok = beta > BETA_ZERO
    X2[:, ok] = L2Y[:, ok] / beta[ok]
    R = Y.T @ Rt
    out = dict(alpha=alpha, beta=beta, U=X1, V=X2, R=R)
    out.update(quantities(alpha, beta))
    return out

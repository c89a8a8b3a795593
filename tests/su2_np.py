"""Independent test-side arithmetic on SU(2) link fields as 2x2 complex
matrices (numpy).  Written from the textbook definitions, not from either
implementation under test, so that it can pin both:

  U = u0 I + i (u1 s1 + u2 s2 + u3 s3)          (Eq. (4))
  U_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag      (Eq. (3))
  S_W = beta sum_x sum_{mu<nu} [1 - (1/2) Tr U_mu,nu(x)]          (Eq. (2))

Link arrays are [V, 4, 4] (site lex, direction, component) with
lex = x0 + L0*(x1 + L1*(x2 + L2*x3)); a site array reshaped C-order to
(L3, L2, L1, L0) puts direction mu on axis 3 - mu.
"""
import numpy as np

SIGMA = np.array([[[0, 1], [1, 0]],
                  [[0, -1j], [1j, 0]],
                  [[1, 0], [0, -1]]], dtype=np.complex128)
ID2 = np.eye(2, dtype=np.complex128)


def to_matrix(q):
    """[..., 4] real quaternions -> [..., 2, 2] complex matrices."""
    q = np.asarray(q, dtype=np.float64)
    m = q[..., 0, None, None] * ID2
    for j in range(3):
        m = m + 1j * q[..., j + 1, None, None] * SIGMA[j]
    return m


def from_matrix(m):
    """Inverse of to_matrix for matrices of the form u0 I + i s.u."""
    u0 = 0.5 * np.real(m[..., 0, 0] + m[..., 1, 1])
    u3 = 0.5 * np.imag(m[..., 0, 0] - m[..., 1, 1])
    u1 = 0.5 * np.imag(m[..., 0, 1] + m[..., 1, 0])
    u2 = 0.5 * np.real(m[..., 0, 1] - m[..., 1, 0])
    return np.stack([u0, u1, u2, u3], axis=-1)


def dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def field(U, dims):
    """[V,4,4] links -> list over mu of [L3,L2,L1,L0,2,2] matrix fields."""
    L0, L1, L2, L3 = dims
    M = to_matrix(np.asarray(U, dtype=np.float64))
    return [M[:, mu].reshape(L3, L2, L1, L0, 2, 2) for mu in range(4)]


def shift(F, mu, step=1):
    """F(x + step*mu) as a field on x (periodic)."""
    return np.roll(F, -step, axis=3 - mu)


def plaquette_fields(U, dims):
    """dict (mu,nu) -> (1/2) Re Tr U_mu,nu(x) over the lattice."""
    F = field(U, dims)
    out = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = F[mu] @ shift(F[nu], mu) @ dag(shift(F[mu], nu)) @ dag(F[nu])
            out[(mu, nu)] = 0.5 * np.real(np.trace(P, axis1=-2, axis2=-1))
    return out


def plaquette(U, dims):
    """(P, P_spatial, P_temporal)."""
    pf = plaquette_fields(U, dims)
    ps = np.mean([pf[k].mean() for k in pf if k[1] != 3])
    pt = np.mean([pf[k].mean() for k in pf if k[1] == 3])
    return np.array([0.5 * (ps + pt), ps, pt])


def wilson_action(U, dims, beta):
    pf = plaquette_fields(U, dims)
    return beta * sum(np.sum(1.0 - v) for v in pf.values())


def staple_fields(U, dims):
    """list over mu of [L3,L2,L1,L0,2,2]: sum over the six plaquettes through
    U_mu(x) of the other three links, oriented so Re Tr(U W^dag)/2 is the sum
    of those plaquettes' (1/2)Tr."""
    F = field(U, dims)
    W = []
    for mu in range(4):
        acc = np.zeros_like(F[0])
        for nu in range(4):
            if nu == mu:
                continue
            acc = acc + F[nu] @ shift(F[mu], nu) @ dag(shift(F[nu], mu))
            Fm = shift(F[nu], nu, -1)  # U_nu(x - nu)
            acc = acc + dag(Fm) @ shift(F[mu], nu, -1) @ shift(shift(F[nu], mu), nu, -1)
        W.append(acc)
    return W


def staples(U, dims):
    """[V, 4, 4] staple quaternions (the staple sum is a real multiple of an
    SU(2) matrix, so it has a quaternion form)."""
    W = staple_fields(U, dims)
    V = int(np.prod(dims))
    return np.stack([from_matrix(W[mu]).reshape(V, 4) for mu in range(4)], axis=1)


def polyakov(U, dims):
    F = field(U, dims)[3]
    L3 = dims[3]
    P = np.broadcast_to(ID2, F.shape[1:]).copy()
    for t in range(L3):
        P = P @ F[t]
    return float(np.mean(0.5 * np.real(np.trace(P, axis1=-2, axis2=-1))))


def gauge_transform(U, dims, G):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag with G [V,4] unit quaternions."""
    L0, L1, L2, L3 = dims
    g = to_matrix(G).reshape(L3, L2, L1, L0, 2, 2)
    F = field(U, dims)
    V = int(np.prod(dims))
    out = np.zeros((V, 4, 4))
    for mu in range(4):
        Fm = g @ F[mu] @ dag(shift(g, mu))
        out[:, mu] = from_matrix(Fm).reshape(V, 4)
    return out

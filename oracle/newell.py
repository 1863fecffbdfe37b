"""Cell-averaged demagnetising tensor and the demag field, plain FP64.

TEST INFRASTRUCTURE ONLY.  Part of the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.

Definition used (the paper switches dipolar interactions off in its own
benchmarks, Sec. IV; the demag term is the standard micromagnetic one):

    B_d(i) = -mu0 * sum_j N(r_i - r_j) . (Ms * G_j * m_j)

with N the tensor of two uniformly magnetised cuboid cells averaged over the
target cell,

    N_ab(R) = 1/(4 pi V) * Int_{[-d,d]^3} Lambda(s) K_ab(R + s) ds,
    Lambda(s) = prod_c (d_c - |s_c|),   K_ab(r) = (delta_ab r^2 - 3 r_a r_b)/r^5.

It is evaluated in closed form (Newell, Williams & Dunlop, J. Geophys. Res.
98, 9551 (1993): the f and g functions and their 27-point second
differences) for |R| < 6 max(d), and by tensor-product Gauss-Legendre
quadrature of the integral above (two panels per axis, split at the kink of
Lambda; 6, 4 or 3 points per panel for |R| below 12, below 40 and beyond, in
cells) where the closed form loses digits to cancellation.  Both pieces are
accurate to about 1e-11 relative.
"""
import numpy as np

MU0 = 4e-7 * np.pi
FAR_CELLS = 6.0


def _safe_div(num, den):
    ok = den != 0
    return np.where(ok, num / np.where(ok, den, 1.0), 0.0)


def newell_f(x, y, z):
    """Newell's f(x, y, z); f is even in each argument."""
    x = np.abs(x); y = np.abs(y); z = np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t1 = 0.5 * y * (z2 - x2) * np.arcsinh(_safe_div(y, np.sqrt(x2 + z2)))
    t2 = 0.5 * z * (y2 - x2) * np.arcsinh(_safe_div(z, np.sqrt(x2 + y2)))
    t3 = -x * y * z * np.arctan(_safe_div(y * z, x * R))
    t4 = (2.0 * x2 - y2 - z2) * R / 6.0
    return t1 + t2 + t3 + t4


def newell_g(x, y, z):
    """Newell's g(x, y, z); g is odd in x and in y, even in z."""
    sx = np.sign(x); sy = np.sign(y)
    x = np.abs(x); y = np.abs(y); z = np.abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    t1 = x * y * z * np.arcsinh(_safe_div(z, np.sqrt(x2 + y2)))
    t2 = y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(_safe_div(x, np.sqrt(y2 + z2)))
    t3 = x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(_safe_div(y, np.sqrt(x2 + z2)))
    t4 = -z2 * z / 6.0 * np.arctan(_safe_div(x * y, z * R))
    t5 = -z * y2 / 2.0 * np.arctan(_safe_div(x * z, y * R))
    t6 = -z * x2 / 2.0 * np.arctan(_safe_div(y * z, x * R))
    t7 = -x * y * R / 3.0
    return sx * sy * (t1 + t2 + t3 + t4 + t5 + t6 + t7)


def _second_difference(fun, X, Y, Z, dx, dy, dz):
    """sum over offsets in {-1,0,1}^3 of prod w(o) * fun(X+o dx, ...), with
    w(0) = 2, w(+-1) = -1, divided by 4 pi dx dy dz."""
    w = {-1: -1.0, 0: 2.0, 1: -1.0}
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                acc = acc + w[i] * w[j] * w[k] * fun(X + i * dx, Y + j * dy, Z + k * dz)
    return acc / (4.0 * np.pi * dx * dy * dz)


def tensor_exact(X, Y, Z, dx, dy, dz):
    """Closed-form (Newell) tensor at displacement (X, Y, Z).

    Returns the six components (xx, yy, zz, xy, xz, yz)."""
    X = np.asarray(X, float); Y = np.asarray(Y, float); Z = np.asarray(Z, float)
    nxx = _second_difference(newell_f, X, Y, Z, dx, dy, dz)
    nyy = _second_difference(newell_f, Y, X, Z, dy, dx, dz)
    nzz = _second_difference(newell_f, Z, Y, X, dz, dy, dx)
    nxy = _second_difference(newell_g, X, Y, Z, dx, dy, dz)
    nxz = _second_difference(newell_g, X, Z, Y, dx, dz, dy)
    nyz = _second_difference(newell_g, Y, Z, X, dy, dz, dx)
    return np.stack([nxx, nyy, nzz, nxy, nxz, nyz])


def _gauss_hat_nodes(d, n):
    """Nodes and weights on [-d, d] for the weight (d - |s|), two panels."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    # panel [0, d]: s = d/2 (xg + 1)
    s_pos = 0.5 * d * (xg + 1.0)
    w_pos = 0.5 * d * wg * (d - s_pos)
    s = np.concatenate([-s_pos, s_pos])
    w = np.concatenate([w_pos, w_pos])
    return s, w


def _far_order(r_cells):
    # Gauss points per panel: keeps the quadrature error near 1e-11 relative
    return np.where(r_cells < 12.0, 6, np.where(r_cells < 40.0, 4, 3))


def tensor_far(X, Y, Z, dx, dy, dz, n):
    """Quadrature of the hat-weighted dipole kernel, n Gauss points per panel."""
    X = np.asarray(X, float).ravel(); Y = np.asarray(Y, float).ravel(); Z = np.asarray(Z, float).ravel()
    sx, wx = _gauss_hat_nodes(dx, n)
    sy, wy = _gauss_hat_nodes(dy, n)
    sz, wz = _gauss_hat_nodes(dz, n)
    out = np.zeros((6, X.size))
    V = dx * dy * dz
    for a, wa in zip(sx, wx):
        for b, wb in zip(sy, wy):
            for c, wc in zip(sz, wz):
                rx, ry, rz = X + a, Y + b, Z + c
                r2 = rx * rx + ry * ry + rz * rz
                inv5 = 1.0 / (r2 * r2 * np.sqrt(r2))
                w = wa * wb * wc * inv5
                out[0] += w * (r2 - 3.0 * rx * rx)
                out[1] += w * (r2 - 3.0 * ry * ry)
                out[2] += w * (r2 - 3.0 * rz * rz)
                out[3] += w * (-3.0 * rx * ry)
                out[4] += w * (-3.0 * rx * rz)
                out[5] += w * (-3.0 * ry * rz)
    return out / (4.0 * np.pi * V)


def tensor(X, Y, Z, dx, dy, dz):
    """Demag tensor at displacements (X, Y, Z) (arrays, metres): closed form
    near, quadrature far.  Shape (6,) + broadcast shape."""
    X, Y, Z = np.broadcast_arrays(np.asarray(X, float), np.asarray(Y, float), np.asarray(Z, float))
    shape = X.shape
    X = X.ravel(); Y = Y.ravel(); Z = Z.ravel()
    r_cells = np.sqrt(X * X + Y * Y + Z * Z) / max(dx, dy, dz)
    out = np.zeros((6, X.size))
    near = r_cells < FAR_CELLS
    if near.any():
        out[:, near] = tensor_exact(X[near], Y[near], Z[near], dx, dy, dz)
    far = ~near
    if far.any():
        order = _far_order(r_cells)
        for n in (6, 4, 3):
            sel = far & (order == n)
            if sel.any():
                idx = np.nonzero(sel)[0]
                for lo in range(0, idx.size, 65536):
                    part = idx[lo:lo + 65536]
                    out[:, part] = tensor_far(X[part], Y[part], Z[part], dx, dy, dz, n)
    return out.reshape((6,) + shape)


def padded_size(n):
    """FFT length for a linear convolution over n cells (power of two, >= 2n)."""
    if n == 1:
        return 1
    p = 1
    while p < 2 * n:
        p *= 2
    return p


# parity of each component (xx, yy, zz, xy, xz, yz) under X -> -X, Y -> -Y, Z -> -Z
PARITY = np.array([[1, 1, 1], [1, 1, 1], [1, 1, 1], [-1, -1, 1], [-1, 1, -1], [1, -1, -1]], float)


def padded_kernel(grid, cell):
    """Real-space kernel on the zero-padded grid, components (xx, yy, zz, xy,
    xz, yz), array shape (6, Pz, Py, Px); displacement d is stored at index
    d mod P for |d| < n.  The tensor is evaluated on displacements >= 0 and
    mirrored with the parity of each component."""
    nx, ny, nz = grid
    dx, dy, dz = cell
    px, py, pz = padded_size(nx), padded_size(ny), padded_size(nz)
    Zg, Yg, Xg = np.meshgrid(np.arange(nz) * dz, np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    octant = tensor(Xg, Yg, Zg, dx, dy, dz)                  # (6, nz, ny, nx)
    K = np.zeros((6, pz, py, px))
    ix = np.arange(-(nx - 1), nx)
    iy = np.arange(-(ny - 1), ny)
    iz = np.arange(-(nz - 1), nz)
    vals = octant[:, np.abs(iz)[:, None, None], np.abs(iy)[None, :, None], np.abs(ix)[None, None, :]]
    sx = np.where(ix < 0, PARITY[:, 0:1], 1.0)[:, None, None, :]
    sy = np.where(iy < 0, PARITY[:, 1:2], 1.0)[:, None, :, None]
    sz = np.where(iz < 0, PARITY[:, 2:3], 1.0)[:, :, None, None]
    K[:, (iz % pz)[:, None, None], (iy % py)[None, :, None], (ix % px)[None, None, :]] = vals * sx * sy * sz
    return K


def kernel_spectrum(grid, cell):
    """rfftn of the padded kernel over (z, y, x): complex (6, Pz, Py, Px//2+1)."""
    K = padded_kernel(grid, cell)
    return np.fft.rfftn(K, axes=(1, 2, 3))


def demag_field_fft(M, grid, cell, spectrum=None):
    """H = -N * M by zero-padded FFT convolution.  M: (3, nz, ny, nx) in A/m.
    Returns H in A/m (multiply by mu0 for tesla)."""
    nx, ny, nz = grid
    if spectrum is None:
        spectrum = kernel_spectrum(grid, cell)
    pz, py = spectrum.shape[1], spectrum.shape[2]
    px = padded_size(nx)
    Mh = np.fft.rfftn(M, s=(pz, py, px), axes=(1, 2, 3))
    xx, yy, zz, xy, xz, yz = spectrum
    Hx = xx * Mh[0] + xy * Mh[1] + xz * Mh[2]
    Hy = xy * Mh[0] + yy * Mh[1] + yz * Mh[2]
    Hz = xz * Mh[0] + yz * Mh[1] + zz * Mh[2]
    H = np.fft.irfftn(np.stack([Hx, Hy, Hz]), s=(pz, py, px), axes=(1, 2, 3))
    return -H[:, :nz, :ny, :nx]


def demag_field_direct(M, grid, cell):
    """H = -N * M by the O(n^2) direct sum over all cell pairs (small grids)."""
    nx, ny, nz = grid
    dx, dy, dz = cell
    zi, yi, xi = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.stack([xi.ravel(), yi.ravel(), zi.ravel()], axis=1)
    Mf = M.reshape(3, -1)
    H = np.zeros_like(Mf)
    for t in range(pos.shape[0]):
        d = pos[t][None, :] - pos
        N = tensor(d[:, 0] * dx, d[:, 1] * dy, d[:, 2] * dz, dx, dy, dz)
        xx, yy, zz, xy, xz, yz = N
        H[0, t] = -(xx @ Mf[0] + xy @ Mf[1] + xz @ Mf[2])
        H[1, t] = -(xy @ Mf[0] + yy @ Mf[1] + yz @ Mf[2])
        H[2, t] = -(xz @ Mf[0] + yz @ Mf[1] + zz @ Mf[2])
    return H.reshape(M.shape)


def mean_tensor(geometry, cell):
    """Volume-averaged tensor of a body: (1/N_geo) sum_i sum_j N(r_i - r_j),
    as a 3x3 matrix; geometry is a boolean (nz, ny, nx) mask."""
    nz, ny, nx = geometry.shape
    M = np.zeros((3, 3, nz, ny, nx))
    out = np.zeros((3, 3))
    G = geometry.astype(float)
    for c in range(3):
        Mc = np.zeros((3, nz, ny, nx))
        Mc[c] = G
        H = demag_field_fft(Mc, (nx, ny, nz), cell)
        for r in range(3):
            out[r, c] = -(H[r] * G).sum() / G.sum()
    return out

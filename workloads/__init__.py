"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays out shapes.  It holds none of
the method's arithmetic (no decoder, no derivative, no PDE update, no
inversion), so the CPU oracle and the HIP path can both consume its output
without sharing any computation.

Every generator takes an explicit integer seed and draws from
``numpy.random.Generator(PCG64(seed))`` in a fixed order, so a (seed, shape)
pair always produces the same arrays.  Weights are drawn and returned as
float32 (the precision the decoder parameters are stored in); consumers widen
them as they need.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

Layer = Tuple[np.ndarray, np.ndarray]  # (W[n_out, n_in], b[n_out]), float32


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def layer_sizes(m: int, r: int, d: int, width: int, depth: int) -> List[int]:
    """Unit counts n_0..n_{depth+1}: input [x; q], `depth` hidden layers, output."""
    return [m + r] + [width] * depth + [d]


def xavier_mlp(gen: np.random.Generator, m: int, r: int, d: int, width: int,
               depth: int, bias_scale: float = 0.0) -> List[Layer]:
    """Xavier/Glorot-uniform weights, drawn layer by layer.

    W ~ U(-a, a) with a = sqrt(6 / (fan_in + fan_out)) (gain 1).  Biases are
    zero by default (the Glorot initialisation convention); ``bias_scale > 0``
    draws them from U(-bias_scale, bias_scale) instead, which the parity tests
    use so that every bias path carries a non-zero value.
    """
    sizes = layer_sizes(m, r, d, width, depth)
    layers: List[Layer] = []
    for n_in, n_out in zip(sizes[:-1], sizes[1:]):
        a = np.sqrt(6.0 / (n_in + n_out))
        W = gen.uniform(-a, a, size=(n_out, n_in)).astype(np.float32)
        if bias_scale > 0:
            b = gen.uniform(-bias_scale, bias_scale, size=n_out).astype(np.float32)
        else:
            b = np.zeros(n_out, dtype=np.float32)
        layers.append((W, b))
    return layers


def siren_mlp(gen: np.random.Generator, m: int, r: int, d: int, width: int,
              depth: int, omega0: float = 30.0) -> List[Layer]:
    """SIREN initialisation (Sitzmann et al. 2020, the paper's default
    omega_0 = 30), drawn layer by layer, with omega_0 folded into the sine
    layers' weights and biases (the network computes sin(W a + b)):
    first layer W ~ omega_0 U(-1/n_in, 1/n_in), hidden layers
    W ~ U(-sqrt(6/n_in), sqrt(6/n_in)), biases of sine layers
    omega_0 U(-1/sqrt(n_in), 1/sqrt(n_in)); the linear output layer
    W ~ U(-sqrt(6/n_in)/omega_0, sqrt(6/n_in)/omega_0), b ~ U(-1/sqrt(n_in), 1/sqrt(n_in))."""
    sizes = layer_sizes(m, r, d, width, depth)
    layers: List[Layer] = []
    last = len(sizes) - 2
    for l, (n_in, n_out) in enumerate(zip(sizes[:-1], sizes[1:])):
        if l == 0:
            a = omega0 / n_in
        elif l < last:
            a = np.sqrt(6.0 / n_in)
        else:
            a = np.sqrt(6.0 / n_in) / omega0
        W = gen.uniform(-a, a, size=(n_out, n_in)).astype(np.float32)
        bb = 1.0 / np.sqrt(n_in) * (omega0 if l < last else 1.0)
        b = gen.uniform(-bb, bb, size=n_out).astype(np.float32)
        layers.append((W, b))
    return layers


def uniform_points(gen: np.random.Generator, n: int, m: int,
                   lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return gen.uniform(lo, hi, size=(n, m)).astype(np.float32)


def grid_points_2d(nx: int, ny: int) -> np.ndarray:
    """Nodes of a uniform (nx x ny) grid on the closed unit square, row-major
    over (x-index, y-index); includes the boundary nodes."""
    xs = np.linspace(0.0, 1.0, nx)
    ys = np.linspace(0.0, 1.0, ny)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float32)


def grid_points_3d(nx: int, ny: int, nz: int, h: float) -> np.ndarray:
    xs = np.arange(nx) * h
    ys = np.arange(ny) * h
    zs = np.arange(nz) * h
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float32)


def box_tet_mesh(nx: int, ny: int, nz: int, h: float, jitter: float = 0.0,
                 gen: np.random.Generator = None) -> Tuple[np.ndarray, np.ndarray]:
    """Tetrahedral mesh of a box of (nx x ny x nz) vertices with spacing h.

    Vertices [nx*ny*nz, 3] float32 in the order of ``grid_points_3d``
    (index (i*ny + j)*nz + k); each cube of 8 neighbouring vertices is split
    into six tetrahedra that share its diagonal from corner (0,0,0) to
    (1,1,1), one for each order in which the path between them steps along
    the three axes; tets [6 (nx-1)(ny-1)(nz-1), 4] int32, listed cube by cube
    with the four vertices in path order.  ``jitter > 0`` moves every vertex
    not on the boundary by U(-jitter h, jitter h) per axis (drawn from
    ``gen``), so the tetrahedra differ in shape and size."""
    X = grid_points_3d(nx, ny, nz, h).astype(np.float64)
    if jitter > 0:
        idx = np.arange(nx * ny * nz)
        i, j, k = idx // (ny * nz), (idx // nz) % ny, idx % nz
        inner = (i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)
        X[inner] += gen.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    orders = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    tets = []
    for c in base:
        for order in orders:
            p = c.copy()
            path = [p.copy()]
            for ax in order:
                p[ax] += 1
                path.append(p.copy())
            tets.append([(a * ny + b) * nz + e for a, b, e in path])
    return X.astype(np.float32), np.asarray(tets, dtype=np.int32)


# --------------------------------------------------------------------------
# Workload recipes.  Each returns plain arrays; none evaluates the method.
# --------------------------------------------------------------------------

@dataclass
class Heat1D:
    """1D heat, nu = 0.5 on [0, 1], Dirichlet 0; decoder (x, q in R^3) ->
    5 ELU layers of width 32 -> 1; 20 samples y_j = j/21; dt = 1e-5."""
    seed: int = 0
    nu: float = 0.5
    dt: float = 1e-5
    steps: int = 1000
    m: int = 1
    r: int = 3
    d: int = 1
    width: int = 32
    depth: int = 5
    n_samples: int = 20
    max_iter: int = 5
    ic: np.ndarray = field(init=False)
    layers: List[Layer] = field(init=False)
    samples: np.ndarray = field(init=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.ic = g.uniform(-1.0, 1.0, size=3)               # a_k, k = 1..3
        self.layers = xavier_mlp(g, self.m, self.r, self.d, self.width, self.depth)
        j = np.arange(1, self.n_samples + 1)
        self.samples = (j / (self.n_samples + 1.0)).reshape(-1, 1).astype(np.float32)


@dataclass
class Heat2D:
    """2D heat on the unit square, 256 x 256 grid, diffusivity mu ~ U(0.1, 1);
    decoder (x in R^2, q in R^8) -> 5 ELU layers of width 128 -> 1;
    full-field decode at the 65,536 grid nodes and derivatives at 2,000
    samples drawn uniformly in (0, 1)^2."""
    seed: int = 0
    grid: int = 256
    n_samples: int = 2000
    m: int = 2
    r: int = 8
    d: int = 1
    width: int = 128
    depth: int = 5
    dt: float = 1e-4
    bias_scale: float = 0.0
    mu: float = field(init=False)
    ic: np.ndarray = field(init=False)
    layers: List[Layer] = field(init=False)
    samples: np.ndarray = field(init=False)
    q0: np.ndarray = field(init=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.mu = float(g.uniform(0.1, 1.0))
        self.ic = g.uniform(-1.0, 1.0, size=(3, 3))          # a_kl, k, l = 1..3
        self.layers = xavier_mlp(g, self.m, self.r, self.d, self.width, self.depth,
                                 self.bias_scale)
        self.samples = uniform_points(g, self.n_samples, self.m)
        self.q0 = g.uniform(-1.0, 1.0, size=self.r)

    @property
    def nodes(self) -> np.ndarray:
        return grid_points_2d(self.grid, self.grid)


@dataclass
class Elastic3D:
    """Neo-Hookean bar of 64 x 16 x 16 material points (spacing h = 1/15),
    lambda = 1e4, mu = 4e3, rho0 = 1000, gravity (0, 0, -9.81); decoder
    (X in R^3, q in R^16) -> 6 ELU layers of width 256 -> 3 (displacement),
    Xavier-uniform with the output layer scaled by out_scale; 500 samples
    drawn from the nodes; the samples on the face X_1 = 0 are clamped."""
    seed: int = 0
    nx: int = 64
    ny: int = 16
    nz: int = 16
    n_samples: int = 500
    m: int = 3
    r: int = 16
    d: int = 3
    width: int = 256
    depth: int = 6
    lam: float = 1e4
    mu: float = 4e3
    rho0: float = 1000.0
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)
    dt: float = 1e-3
    out_scale: float = 1e-2
    layers: List[Layer] = field(init=False)
    sample_idx: np.ndarray = field(init=False)
    q0: np.ndarray = field(init=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.layers = xavier_mlp(g, self.m, self.r, self.d, self.width, self.depth)
        # displacements of order out_scale: small strains, det F near 1
        W, b = self.layers[-1]
        self.layers[-1] = ((W * self.out_scale).astype(np.float32), (b * self.out_scale).astype(np.float32))
        n_nodes = self.nx * self.ny * self.nz
        self.sample_idx = np.sort(g.choice(n_nodes, size=self.n_samples, replace=False))
        self.q0 = g.uniform(-0.1, 0.1, size=self.r)

    @property
    def h(self) -> float:
        return 1.0 / 15.0

    @property
    def nodes(self) -> np.ndarray:
        return grid_points_3d(self.nx, self.ny, self.nz, self.h)


@dataclass
class Corotated3D:
    """Falling bar with finite-element forces: the bar of 64 x 16 x 16
    vertices (spacing h = 1/15) as a tetrahedral mesh (``box_tet_mesh``, six
    tetrahedra per cube, interior vertices jittered by up to 0.15 h);
    corotated elasticity with the paper's gravity-impact parameters
    mu ~ U(6e4, 7e4) per instance and lam = 0, rho0 = 1000, gravity
    (0, 0, -9.81), dt = 1e-3; decoder as the neo-Hookean bar's (Xavier-uniform,
    output scaled by out_scale); n_samples sample vertices per instance drawn
    without replacement, none clamped (the body falls freely)."""
    seed: int = 0
    nx: int = 64
    ny: int = 16
    nz: int = 16
    jitter: float = 0.15
    n_samples: int = 500
    n_inst: int = 1
    m: int = 3
    r: int = 16
    d: int = 3
    width: int = 256
    depth: int = 6
    lam: float = 0.0
    mu_range: Tuple[float, float] = (6e4, 7e4)
    rho0: float = 1000.0
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)
    dt: float = 1e-3
    out_scale: float = 1e-2
    layers: List[Layer] = field(init=False)
    X: np.ndarray = field(init=False)
    tets: np.ndarray = field(init=False)
    samples: List[np.ndarray] = field(init=False)
    mu: np.ndarray = field(init=False)
    q0: np.ndarray = field(init=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.layers = xavier_mlp(g, self.m, self.r, self.d, self.width, self.depth)
        W, b = self.layers[-1]
        self.layers[-1] = ((W * self.out_scale).astype(np.float32), (b * self.out_scale).astype(np.float32))
        self.X, self.tets = box_tet_mesh(self.nx, self.ny, self.nz, 1.0 / 15.0, self.jitter, g)
        n = self.X.shape[0]
        self.samples = [np.sort(g.choice(n, size=self.n_samples, replace=False)) for _ in range(self.n_inst)]
        self.mu = g.uniform(*self.mu_range, size=self.n_inst)
        self.q0 = g.uniform(-0.1, 0.1, size=(self.n_inst, self.r))


@dataclass
class Batched2D:
    """Ragged batch of 2D heat instances: mu_i ~ U(0.1, 1), per-instance sample
    counts S_i ~ U{s_min..s_max}, samples drawn without replacement from the
    interior nodes of a (grid x grid) node lattice; r = 8, width 128."""
    seed: int = 0
    n_inst: int = 512
    s_min: int = 200
    s_max: int = 2000
    grid: int = 128
    m: int = 2
    r: int = 8
    d: int = 1
    width: int = 128
    depth: int = 5
    dt: float = 1e-4
    mu: np.ndarray = field(init=False)
    counts: np.ndarray = field(init=False)
    offsets: np.ndarray = field(init=False)
    samples: np.ndarray = field(init=False)
    layers: List[Layer] = field(init=False)
    q0: np.ndarray = field(init=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.mu = g.uniform(0.1, 1.0, size=self.n_inst)
        self.counts = g.integers(self.s_min, self.s_max + 1, size=self.n_inst)
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        n_int = (self.grid - 2) ** 2
        h = 1.0 / (self.grid - 1)
        pts = []
        for s in self.counts:
            idx = g.choice(n_int, size=int(s), replace=False)
            ix = 1 + idx // (self.grid - 2)
            iy = 1 + idx % (self.grid - 2)
            pts.append(np.stack([ix * h, iy * h], axis=1))
        self.samples = np.concatenate(pts, axis=0).astype(np.float32)
        self.layers = xavier_mlp(g, self.m, self.r, self.d, self.width, self.depth)
        self.q0 = g.uniform(-1.0, 1.0, size=(self.n_inst, self.r))


@dataclass
class Train2D:
    """Decoder training on 2D heat snapshots: unit square, 128 x 128 nodes,
    n_mu = 40 training diffusivities mu ~ U(0.1, 1) (and 4 held-out ones),
    one initial field shared by every mu, snapshots at 5 times in [0, 0.05]
    (200 snapshots); encoder 16,384 -> 256 -> 8, decoder (x in R^2, q in R^8)
    -> 5 ELU layers of width 128 -> 1; batches of 16 snapshots, Adam lr 1e-3.
    The initial field is a window sin(pi x) sin(pi y) times a sum of Gaussian
    bumps (centres in [0.25, 0.75]^2, widths U(0.06, 0.12), amplitudes
    +-U(0.5, 1)), zero on the boundary.  The reduced-order rollout steps
    with dt = 1e-4 at n_samples interior nodes drawn without replacement."""
    seed: int = 0
    grid: int = 128
    n_mu: int = 40
    n_mu_test: int = 4
    times: Tuple[float, ...] = (0.0, 0.0125, 0.025, 0.0375, 0.05)
    dt_fd: float = 1e-5
    n_bumps: int = 4
    batch: int = 16
    lr: float = 1e-3
    enc_hidden: int = 256
    m: int = 2
    r: int = 8
    d: int = 1
    width: int = 128
    depth: int = 5
    dt: float = 1e-4
    n_samples: int = 500
    mu: np.ndarray = field(init=False)
    mu_test: np.ndarray = field(init=False)
    centres: np.ndarray = field(init=False)
    widths: np.ndarray = field(init=False)
    amps: np.ndarray = field(init=False)
    layers: List[Layer] = field(init=False)
    enc_layers: List[Layer] = field(init=False)
    sample_idx: np.ndarray = field(init=False)

    def __post_init__(self):
        g = rng(self.seed)
        self.mu = g.uniform(0.1, 1.0, size=self.n_mu)
        self.mu_test = g.uniform(0.1, 1.0, size=self.n_mu_test)
        self.centres = g.uniform(0.25, 0.75, size=(self.n_bumps, 2))
        self.widths = g.uniform(0.06, 0.12, size=self.n_bumps)
        self.amps = g.uniform(0.5, 1.0, size=self.n_bumps) * g.choice([-1.0, 1.0], size=self.n_bumps)
        self.layers = xavier_mlp(g, self.m, self.r, self.d, self.width, self.depth)
        self.enc_layers = xavier_mlp(g, self.grid * self.grid, 0, self.r, self.enc_hidden, 1)
        n_int = (self.grid - 2) ** 2
        idx = g.choice(n_int, size=self.n_samples, replace=False)
        self.sample_idx = np.sort((1 + idx // (self.grid - 2)) * self.grid + 1 + idx % (self.grid - 2))

    @property
    def nodes(self) -> np.ndarray:
        return grid_points_2d(self.grid, self.grid)

    @property
    def dx(self) -> float:
        return 1.0 / (self.grid - 1)

    def initial_field(self) -> np.ndarray:
        """The initial field on the nodes, [grid, grid] float64 (index [i_x][i_y])."""
        xs = np.linspace(0.0, 1.0, self.grid)
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        u = np.zeros_like(X)
        for (cx, cy), w, a in zip(self.centres, self.widths, self.amps):
            u += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * w * w))
        u *= np.sin(np.pi * X) * np.sin(np.pi * Y)
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
        return u

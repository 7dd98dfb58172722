"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method: it only draws particle positions
and complex charges.  It is shared by the tests, bench.py and the oracle checks.

Layered-medium conventions: ``d`` lists the L interfaces top to bottom (strictly
decreasing); ``k`` lists the L+1 real wavenumbers, layer 0 on top (z > d[0]),
layer l between d[l] (below) and d[l-1] (above).

The three-layer geometry (interfaces z = 0, -1.2) follows the paper's Section 4
test problem; the unit cubes centred at (0,0,0.6), (0,0,-0.6), (0,0,-1.8) keep
every particle at least 0.1 away from an interface.  The paper's own irregular
domains are replaced by these cubes.
"""
import numpy as np

THREE_LAYER_D = (0.0, -1.2)
THREE_LAYER_K = (0.8, 1.5, 2.0)
THREE_LAYER_CENTERS = (0.6, -0.6, -1.8)


def split_even(n, parts):
    """n split into `parts` counts, the remainder going to the top layers."""
    base, rem = divmod(n, parts)
    return [base + (1 if i < rem else 0) for i in range(parts)]


def layered_cubes(d, k, counts, centers, side=1.0, seed=0, shuffle=False):
    """Uniform particles in axis-aligned cubes (one per layer) with complex charges
    whose real and imaginary parts are uniform on [-1, 1]."""
    rng = np.random.default_rng(seed)
    xs, ys, zs, ls = [], [], [], []
    for l, (n, c) in enumerate(zip(counts, centers)):
        xs.append(rng.uniform(-0.5, 0.5, n) * side)
        ys.append(rng.uniform(-0.5, 0.5, n) * side)
        zs.append(c + rng.uniform(-0.5, 0.5, n) * side)
        ls.append(np.full(n, l, dtype=np.int32))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    z = np.concatenate(zs)
    layer = np.concatenate(ls).astype(np.int32)
    nt = len(x)
    q = rng.uniform(-1.0, 1.0, nt) + 1j * rng.uniform(-1.0, 1.0, nt)
    if shuffle:
        perm = rng.permutation(nt)
        x, y, z, layer, q = x[perm], y[perm], z[perm], layer[perm], q[perm]
    return dict(d=np.array(d, dtype=np.float64), k=np.array(k, dtype=np.float64), x=x, y=y, z=z,
                layer=layer, q=q.astype(np.complex128))


def three_layer_3k(seed=1):
    """Plain FP64 case: 3 layers, 1000 uniform particles per unit cube, p = 5, leaf <= 50."""
    w = layered_cubes(THREE_LAYER_D, THREE_LAYER_K, [1000, 1000, 1000], THREE_LAYER_CENTERS, seed=seed)
    w.update(p=5, leaf=50, name="3-layer cubes, N=3000, p=5, leaf<=50")
    return w


def three_layer_cubes(n=1048576, seed=2, p=8, leaf=256):
    """N = 1,048,576 split evenly over the three unit cubes (each 0.1 clear of the
    interfaces), p = 8.  The leaf bound 256 gives depth-4 layer trees (about 85
    particles per leaf), the fastest of the depths this workload allows."""
    counts = split_even(n, 3)
    w = layered_cubes(THREE_LAYER_D, THREE_LAYER_K, counts, THREE_LAYER_CENTERS, seed=seed)
    w.update(p=p, leaf=leaf, name="3-layer cubes, N=%d, p=%d, leaf<=%d" % (n, p, leaf))
    return w


def small_three_layer(n_per_layer=100, seed=0, p=4, leaf=16, shuffle=False):
    w = layered_cubes(THREE_LAYER_D, THREE_LAYER_K, [n_per_layer] * 3, THREE_LAYER_CENTERS, seed=seed,
                      shuffle=shuffle)
    w.update(p=p, leaf=leaf, name="3-layer cubes, %d per layer" % n_per_layer)
    return w


def batch_three_layer(seed=3, nprob=256, nmin=2048, nmax=65536, p=6, leaf=64):
    """Batching case: independent three-layer problems, interfaces at 0 and -g with
    g uniform on [1.0, 2.0], k per layer uniform on [0.5, 2.5], N log-uniform on
    [nmin, nmax] split evenly over the layers; uniform particles in the top cube
    [-0.5, 0.5]^2 x [0.1, 1.1], a middle cube of side g - 0.2 centred at (0, 0, -g/2)
    (0.1 clear of both interfaces) and the bottom cube [-0.5, 0.5]^2 x [-g-1.1, -g-0.1]."""
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(nprob):
        g = rng.uniform(1.0, 2.0)
        k = rng.uniform(0.5, 2.5, 3)
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        counts = split_even(n, 3)
        sm = g - 0.2
        xs, ys, zs, ls = [], [], [], []
        for l, (c, side, zc) in enumerate(zip(counts, (1.0, sm, 1.0), (0.6, -g / 2, -g - 0.6))):
            xs.append(rng.uniform(-0.5, 0.5, c) * side)
            ys.append(rng.uniform(-0.5, 0.5, c) * side)
            zs.append(zc + rng.uniform(-0.5, 0.5, c) * side)
            ls.append(np.full(c, l, dtype=np.int32))
        q = rng.uniform(-1.0, 1.0, n) + 1j * rng.uniform(-1.0, 1.0, n)
        probs.append(dict(d=np.array([0.0, -g]), k=k, x=np.concatenate(xs), y=np.concatenate(ys),
                          z=np.concatenate(zs), layer=np.concatenate(ls), q=q.astype(np.complex128), p=p, leaf=leaf))
    return probs


FIVE_LAYER_D = (0.0, -0.6, -1.2, -1.8)
FIVE_LAYER_K = (0.5, 1.2, 2.0, 2.8, 3.0)


def five_layer_clusters(n=16777216, seed=5, clusters=8, sigma=0.05, gap=0.05, p=10, leaf=64):
    """Five-layer medium, N split evenly over the layers (remainder to the top); in
    each layer a mixture of `clusters` Gaussian clusters (standard deviation sigma)
    with centres uniform in x, y in [-0.5, 0.5] and z in the layer's admissible band
    (top [0.05, 1.05], middle layers [d_l + gap, d_{l-1} - gap], bottom
    [-2.85, -1.85]); draws outside the layer or closer than `gap` to an interface
    are redrawn.  Complex charges with Re, Im uniform on [-1, 1]."""
    d = np.array(FIVE_LAYER_D)
    rng = np.random.default_rng(seed)
    counts = split_even(n, 5)
    bands = [(0.05, 1.05)] + [(d[l] + gap, d[l - 1] - gap) for l in range(1, 4)] + [(-2.85, -1.85)]
    lo_z = [d[0] + gap] + [d[l] + gap for l in range(1, 4)] + [-np.inf]
    hi_z = [np.inf] + [d[l - 1] - gap for l in range(1, 4)] + [d[3] - gap]
    xs, ys, zs, ls = [], [], [], []
    for l in range(5):
        cx = rng.uniform(-0.5, 0.5, clusters)
        cy = rng.uniform(-0.5, 0.5, clusters)
        cz = rng.uniform(bands[l][0], bands[l][1], clusters)
        want = counts[l]
        px, py, pz = [], [], []
        got = 0
        while got < want:
            m = int((want - got) * 1.3) + 16
            c = rng.integers(0, clusters, m)
            x = cx[c] + sigma * rng.standard_normal(m)
            y = cy[c] + sigma * rng.standard_normal(m)
            z = cz[c] + sigma * rng.standard_normal(m)
            ok = (z > lo_z[l]) & (z < hi_z[l])
            px.append(x[ok]); py.append(y[ok]); pz.append(z[ok])
            got += int(ok.sum())
        xs.append(np.concatenate(px)[:want]); ys.append(np.concatenate(py)[:want]); zs.append(np.concatenate(pz)[:want])
        ls.append(np.full(want, l, dtype=np.int32))
    nt = sum(counts)
    q = rng.uniform(-1.0, 1.0, nt) + 1j * rng.uniform(-1.0, 1.0, nt)
    return dict(d=d, k=np.array(FIVE_LAYER_K), x=np.concatenate(xs), y=np.concatenate(ys), z=np.concatenate(zs),
                layer=np.concatenate(ls), q=q.astype(np.complex128), p=p, leaf=leaf,
                name="5-layer Gaussian clusters, N=%d, p=%d, leaf<=%d" % (nt, p, leaf))


# Ten interfaces, eleven layers 0.6 thick (the paper expects L of about 10 in
# practice, Section 5); wavenumbers rising with depth.
TEN_LAYER_D = tuple(-0.6 * i for i in range(10))
TEN_LAYER_K = tuple(0.5 + 0.25 * i for i in range(11))
TEN_LAYER_CENTERS = (0.3,) + tuple(-0.3 - 0.6 * i for i in range(9)) + (-5.7,)


def ten_layer(n=1048576, seed=10, p=8, leaf=256, side=0.3):
    """Ten-interface stack: N split evenly over the eleven layers, one cube of side
    `side` in each, centred in the layer (top and bottom: 0.3 from their interface),
    so every particle is at least (0.6 - side) / 2 from an interface."""
    w = layered_cubes(TEN_LAYER_D, TEN_LAYER_K, split_even(n, 11), TEN_LAYER_CENTERS, side=side, seed=seed)
    w.update(p=p, leaf=leaf, name="10-interface cubes, N=%d, p=%d, leaf<=%d" % (n, p, leaf))
    return w

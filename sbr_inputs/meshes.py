"""Seeded triangle-mesh generators (geometry only).

Every generator returns ``(V, T)`` with ``V`` a float32 array of shape
``(n_v, 3)`` (metres) and ``T`` an int32 array of shape ``(n_t, 3)`` of vertex
indices.  Geometry is built in float64 and rounded once to float32, so the
float32 mesh is the single definition both sides consume.
"""
import numpy as np


def _finish(V, T):
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float64).astype(np.float32))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.int64).astype(np.int32))
    return V, T


def mesh_area(V, T):
    """Total surface area (float64), used for input sanity checks only."""
    V = V.astype(np.float64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1).sum()


# --------------------------------------------------------------------------
# Sphere: icosahedron refined by edge midpoints, projected on the sphere.
# --------------------------------------------------------------------------
def icosphere(subdivisions=5, radius=1.0):
    """Icosphere: 20*4**s triangles, 10*4**s + 2 vertices.

    Subdivision 5 gives 20,480 triangles and 10,242 vertices.  The base
    icosahedron has vertices (0, +-1, +-g), (+-1, +-g, 0), (+-g, 0, +-1) with
    g the golden ratio, so the first refinement already places vertices on
    the three coordinate axes and the bounding box is exactly [-r, r]^3.
    """
    g = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0),
             (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
             (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    F = list(faces)
    for _ in range(subdivisions):
        cache = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = V[i] + V[j]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    V = np.array(V) * radius
    return _finish(V, F)


# --------------------------------------------------------------------------
# Flat pieces
# --------------------------------------------------------------------------
def _grid_quad(origin, du, dv, nu, nv, vbase=0):
    """Planar parallelogram origin + s*du + t*dv, s,t in [0,1], nu x nv cells,
    two triangles per cell."""
    origin, du, dv = (np.asarray(x, dtype=np.float64) for x in (origin, du, dv))
    s = np.linspace(0.0, 1.0, nu + 1)
    t = np.linspace(0.0, 1.0, nv + 1)
    S, Tt = np.meshgrid(s, t, indexing="ij")
    P = origin + S[..., None] * du + Tt[..., None] * dv
    V = P.reshape(-1, 3)
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1) + vbase
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    T = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return V, T


def plate(a=1.0, b=1.0, nx=8, ny=8, z=0.0):
    """Rectangle [-a/2, a/2] x [-b/2, b/2] in the plane z = const."""
    V, T = _grid_quad((-a / 2, -b / 2, z), (a, 0, 0), (0, b, 0), nx, ny)
    return _finish(V, T)


def duct(length=6.0, width=0.1, height=0.1, n=24):
    """Rectangular duct along +x, open at x = 0 and closed by a plate at
    x = length; walls at y = +-width/2 and z = +-height/2 (an engine-intake
    like cavity: rays entering at an angle bounce between the walls, hit the
    back plate and come out again)."""
    L, w, h = length, width / 2, height / 2
    parts = [((0, -w, -h), (L, 0, 0), (0, 0, 2 * h)),   # y = -w
             ((0, w, -h), (L, 0, 0), (0, 0, 2 * h)),    # y = +w
             ((0, -w, -h), (L, 0, 0), (0, 2 * w, 0)),   # z = -h
             ((0, -w, h), (L, 0, 0), (0, 2 * w, 0)),    # z = +h
             ((L, -w, -h), (0, 2 * w, 0), (0, 0, 2 * h))]  # back plate
    Vs, Ts, nv = [], [], 0
    for i, (o, du, dv) in enumerate(parts):
        V, T = _grid_quad(o, du, dv, n if i < 4 else 2, 2, vbase=nv)
        Vs.append(V)
        Ts.append(T)
        nv += len(V)
    return _finish(np.concatenate(Vs), np.concatenate(Ts))


def dihedral(a=1.0, b=1.0, n=8):
    """90-degree dihedral: faces x=0 (y in [0,a]) and y=0 (x in [0,a]),
    both spanning z in [-b/2, b/2].  Its bisector is phi = 45 deg in the
    x-y plane (theta = 90 deg)."""
    V1, T1 = _grid_quad((0, 0, -b / 2), (0, a, 0), (0, 0, b), n, n)
    V2, T2 = _grid_quad((0, 0, -b / 2), (a, 0, 0), (0, 0, b), n, n, vbase=len(V1))
    return _finish(np.concatenate([V1, V2]), np.concatenate([T1, T2]))


def trihedral(a=1.0, n=16):
    """Square trihedral corner reflector: three a x a faces on the planes
    x=0, y=0, z=0 in the positive octant, each split into n x n squares of
    two triangles (n=16 gives 512 per face, 1,536 in all)."""
    parts = [((0, 0, 0), (0, a, 0), (0, 0, a)),
             ((0, 0, 0), (0, 0, a), (a, 0, 0)),
             ((0, 0, 0), (a, 0, 0), (0, a, 0))]
    Vs, Ts, base = [], [], 0
    for o, du, dv in parts:
        V, T = _grid_quad(o, du, dv, n, n, vbase=base)
        Vs.append(V)
        Ts.append(T)
        base += len(V)
    return _finish(np.concatenate(Vs), np.concatenate(Ts))


def random_triangles(n, seed=0, box=1.0, size=0.1):
    """Triangle soup: n triangles with centres uniform in [-box, box]^3 and
    vertex offsets of scale ``size``."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-box, box, size=(n, 1, 3))
    off = rng.normal(scale=size, size=(n, 3, 3))
    V = (c + off).reshape(-1, 3)
    T = np.arange(3 * n).reshape(n, 3)
    return _finish(V, T)


# --------------------------------------------------------------------------
# Procedural aircraft
# --------------------------------------------------------------------------
def _lathe(xs, rs, nb, center=(0.0, 0.0, 0.0), vbase=0):
    """Surface of revolution about the x axis through ``center``.

    ``xs``/``rs`` give the profile; a ring with r == 0 at either end becomes
    a single pole vertex joined to the next ring by a fan (no zero-area
    triangles)."""
    cy, cz = center[1], center[2]
    beta = np.linspace(0.0, 2.0 * np.pi, nb, endpoint=False)
    V, T, ring_ids = [], [], []
    nxt = vbase
    for x, r in zip(xs, rs):
        if r == 0.0:
            V.append([[x + center[0], cy, cz]])
            ring_ids.append(np.array([nxt]))
            nxt += 1
        else:
            ring = np.stack([np.full(nb, x + center[0]), cy + r * np.cos(beta),
                             cz + r * np.sin(beta)], 1)
            V.append(ring)
            ring_ids.append(np.arange(nxt, nxt + nb))
            nxt += nb
    for r0, r1 in zip(ring_ids[:-1], ring_ids[1:]):
        if len(r0) == 1 and len(r1) == 1:
            continue
        if len(r0) == 1:
            j = np.arange(nb)
            T.append(np.stack([np.full(nb, r0[0]), r1[(j + 1) % nb], r1[j]], 1))
        elif len(r1) == 1:
            j = np.arange(nb)
            T.append(np.stack([r0[j], r0[(j + 1) % nb], np.full(nb, r1[0])], 1))
        else:
            j = np.arange(nb)
            a, b = r0[j], r0[(j + 1) % nb]
            c, d = r1[(j + 1) % nb], r1[j]
            T.append(np.stack([a, b, c], 1))
            T.append(np.stack([a, c, d], 1))
    return np.concatenate(V), np.concatenate(T)


def _lifting_surface(root, span_dir, up_dir, semi_span, c_root, c_tip, sweep_deg,
                     th_root, th_tip, ns, ne, vbase=0):
    """Closed thin lifting surface (wing or fin) with a lens-shaped section.

    The leading edge starts at ``root`` and runs along ``span_dir`` with the
    given sweep (chord along +x goes towards the tail, i.e. -x is forward).
    Upper/lower skins meet at the leading and trailing edges; the tip is
    closed by a strip of triangles between the two skins."""
    root = np.asarray(root, dtype=np.float64)
    span_dir = np.asarray(span_dir, dtype=np.float64)
    up_dir = np.asarray(up_dir, dtype=np.float64)
    chord_dir = np.array([1.0, 0.0, 0.0])
    tan_sw = np.tan(np.radians(sweep_deg))
    eta = np.linspace(0.0, 1.0, ne + 1)
    s = 0.5 - 0.5 * np.cos(np.linspace(0.0, np.pi, ns + 1))   # cosine spacing
    E, S = np.meshgrid(eta, s, indexing="ij")
    chord = c_root + E * (c_tip - c_root)
    th = th_root + E * (th_tip - th_root)
    le = root + (E * semi_span)[..., None] * span_dir + (E * semi_span * tan_sw)[..., None] * chord_dir
    base_pt = le + (S * chord)[..., None] * chord_dir
    half = (0.5 * th * 4.0 * S * (1.0 - S))[..., None] * up_dir
    upper = base_pt + half
    lower = base_pt - half
    Vs, Ts = [], []
    nv_grid = (ne + 1) * (ns + 1)
    idx = np.arange(nv_grid).reshape(ne + 1, ns + 1)
    for k, P in enumerate((upper, lower)):
        off = vbase + k * nv_grid
        Vs.append(P.reshape(-1, 3))
        a = idx[:-1, :-1].ravel() + off
        b = idx[1:, :-1].ravel() + off
        c = idx[1:, 1:].ravel() + off
        d = idx[:-1, 1:].ravel() + off
        # skip the zero-width cells at the leading/trailing edge pinch
        Ts.append(np.stack([a, b, c], 1))
        Ts.append(np.stack([a, c, d], 1))
    # tip cap between upper and lower skins at eta = 1 (interior section points)
    up_tip = idx[-1, :] + vbase
    lo_tip = idx[-1, :] + vbase + nv_grid
    j = np.arange(1, ns - 1)
    Ts.append(np.stack([up_tip[j], lo_tip[j], lo_tip[j + 1]], 1))
    Ts.append(np.stack([up_tip[j], lo_tip[j + 1], up_tip[j + 1]], 1))
    Ts.append(np.array([[up_tip[0], lo_tip[1], up_tip[1]],
                        [up_tip[ns - 1], lo_tip[ns - 1], up_tip[ns]]]))
    return np.concatenate(Vs), np.concatenate(Ts)


def aircraft(seed=0, scale=1.0):
    """Aircraft-like PEC target.

    Ellipsoidal fuselage 15 m long with 1.5 m radius; swept trapezoidal wings
    of 12 m span (0.3 m thick at the root, 0.1 m at the tip); a vertical fin
    and a horizontal tail; two open cylindrical engine inlets (0.6 m radius,
    3 m deep, closed back wall) under the wings.  The nose points to -x.
    ``seed`` perturbs the planform dimensions by a few percent; ``scale``
    multiplies the tessellation density per direction (scale=1 gives about
    1.5 million triangles, scale=0.1 about 15 thousand)."""
    rng = np.random.default_rng(seed)
    j = lambda: 1.0 + 0.03 * rng.uniform(-1.0, 1.0)   # noqa: E731
    res = lambda n: max(4, int(round(n * scale)))       # noqa: E731
    Vs, Ts, base = [], [], 0

    def add(VT):
        nonlocal base
        V, T = VT
        Vs.append(V)
        Ts.append(T)
        base += len(V)

    # fuselage: x = -L/2 cos(a), r = R sin(a); poles at the nose and tail
    L, R = 15.0, 1.5 * j()
    na, nb = res(640), res(500)
    a = np.linspace(0.0, np.pi, na + 1)
    xs = -0.5 * L * np.cos(a)
    rs = R * np.sin(a)
    rs[0] = rs[-1] = 0.0
    add(_lathe(xs, rs, nb, vbase=base))
    # main wings (left/right), leading-edge root at x = -2.5
    c_root, c_tip, sweep = 4.0 * j(), 1.5 * j(), 30.0 * j()
    for sgn in (1.0, -1.0):
        add(_lifting_surface((-2.5, 0.0, -0.3), (0.0, sgn, 0.0), (0.0, 0.0, 1.0),
                             6.0, c_root, c_tip, sweep, 0.3, 0.1,
                             res(180), res(300), vbase=base))
    # horizontal tail
    for sgn in (1.0, -1.0):
        add(_lifting_surface((4.6, 0.0, 0.3), (0.0, sgn, 0.0), (0.0, 0.0, 1.0),
                             2.6 * j(), 1.8, 0.8, 35.0, 0.12, 0.06,
                             res(90), res(120), vbase=base))
    # vertical fin
    add(_lifting_surface((4.0, 0.0, 1.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0),
                         3.0 * j(), 2.6, 1.0, 40.0, 0.18, 0.08,
                         res(100), res(140), vbase=base))
    # engine inlets: open at the front (x = x0 - d/2), back wall at x0 + d/2
    r_in, depth = 0.6, 3.0
    for sgn in (1.0, -1.0):
        x0, y0, z0 = -0.5, sgn * 3.2, -1.2
        n_len, n_rim = res(200), res(280)
        xs = np.linspace(x0 - depth / 2, x0 + depth / 2, n_len + 1)
        rs = np.full_like(xs, r_in)
        V, T = _lathe(xs, rs, n_rim, center=(0.0, y0, z0), vbase=base)
        add((V, T))
        # back wall: disk at x0 + depth/2 made of rings down to a centre pole
        nr = res(60)
        xs = np.full(nr + 1, x0 + depth / 2)
        rs = np.linspace(r_in, 0.0, nr + 1)
        add(_lathe(xs, rs, n_rim, center=(0.0, y0, z0), vbase=base))
    V = np.concatenate(Vs)
    T = np.concatenate(Ts)
    # drop triangles that collapse to zero area at lens pinches (exact
    # duplicate vertices), keeping the mesh free of degenerate facets
    Vd = V[T]
    area2 = np.linalg.norm(np.cross(Vd[:, 1] - Vd[:, 0], Vd[:, 2] - Vd[:, 0]), axis=1)
    T = T[area2 > 1e-12]
    return _finish(V, T)

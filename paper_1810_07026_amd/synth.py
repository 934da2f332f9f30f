"""Seeded synthetic hydrocarbon systems (inputs only, no potential arithmetic).

Every generator returns a dict with ``x`` [n,3] positions (A), ``species``
[n] (0 = C, 1 = H), ``box`` [3] (A), ``periodic`` [3], ``v`` [n,3] (A/fs,
when velocities are requested) and ``meta``.  Geometry: C-C 1.54 A, C-H 1.09
A, tetrahedral angles; these stand in for the paper's polyethylene benchmark
and model problems (Sec. 5.1), which are not available.

Both the GPU tests and the CPU oracle tests draw their inputs from here; the
module holds none of the AIREBO method's arithmetic.
"""
import math

import numpy as np

CC, CH = 1.54, 1.09
TETRA = math.acos(-1.0 / 3.0)          # 109.47 degrees
MASS = (12.011, 1.008)                 # amu
KB = 8.617333262e-5                    # eV/K
MVV2E = 103.642691                     # amu A^2/fs^2 -> eV
SEED0 = 1810070260

# Non-bonded distances when placing atoms (A), by species pair: never below
# the hard floor (keeps every non-bonded pair outside the bonding range), and
# the trial torsion that best clears the soft target is kept.
_HARD = np.array([[2.05, 1.85], [1.85, 1.75]])
_SOFT = np.array([[3.0, 2.5], [2.5, 2.2]])
# Growth at melt density uses a low floor and relies on _relax() afterwards.
_GROW_FLOOR = np.array([[1.7, 1.45], [1.45, 1.3]])
# Non-bonded targets of the relaxation (every pair ends at or above _HARD).
_RELAX = np.array([[2.15, 1.95], [1.95, 1.85]])


def _unit(v):
    return v / np.linalg.norm(v)


def _nerf(a, b, c, bond, angle, torsion):
    """Position of d with |cd| = bond, angle(b,c,d) = angle, dihedral(a,b,c,d) = torsion."""
    bc = _unit(c - b)
    n = _unit(np.cross(b - a, bc))
    m = np.cross(n, bc)
    d2 = np.array([-bond * math.cos(angle), bond * math.sin(angle) * math.cos(torsion),
                   bond * math.sin(angle) * math.sin(torsion)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * n


def _ch2_hydrogens(prev, cur, nxt):
    """Two tetrahedral hydrogens of a CH2 carbon between two backbone carbons."""
    a, b = _unit(prev - cur), _unit(nxt - cur)
    u = -_unit(a + b)
    n = _unit(np.cross(a, b))
    half = TETRA / 2.0
    return [cur + CH * (math.cos(half) * u + math.sin(half) * n),
            cur + CH * (math.cos(half) * u - math.sin(half) * n)]


def _ch3_hydrogens(a, b, c):
    """Three staggered hydrogens on carbon c bonded to b (a: the atom before b)."""
    return [_nerf(a, b, c, CH, TETRA, t) for t in (math.pi, math.pi / 3, -math.pi / 3)]


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def maxwell_velocities(species, T, rng):
    """Gaussian velocities at temperature T, zero net momentum, rescaled to exactly T (3N-3 dof)."""
    m = np.asarray(MASS)[np.asarray(species)]
    n = len(m)
    v = rng.normal(size=(n, 3)) * np.sqrt(KB * T / (m * MVV2E))[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ke = 0.5 * (m[:, None] * v * v).sum() * MVV2E
    if n > 1 and ke > 0:
        v *= math.sqrt(T / (2.0 * ke / ((3 * n - 3) * KB)))
    return v


class _Packer:
    """Cell grid of placed atoms for distance checks in a periodic box."""

    def __init__(self, box, cap, cell=5.6, zwall=None, floor=None):
        self.box = np.asarray(box, float)
        self.floor = _HARD if floor is None else floor
        self.nc = np.maximum(1, np.floor(self.box / cell).astype(int))
        self.cells = {}
        self.x = np.zeros((cap, 3))
        self.s = np.zeros(cap, dtype=np.int32)
        self.chain = np.zeros(cap, dtype=np.int64)
        self.pos = np.zeros(cap, dtype=np.int64)
        self.alive = np.zeros(cap, dtype=bool)
        self.free = []
        self.n = 0
        self.zwall = zwall

    def _key(self, p):
        f = np.floor((p % self.box) / self.box * self.nc).astype(int) % self.nc
        return (int(f[0]), int(f[1]), int(f[2]))

    def near(self, p):
        """Indices of placed atoms in the 27 cells around p."""
        k = self._key(p)
        seen = set()
        idx = []
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for c in (-1, 0, 1):
                    q = ((k[0] + a) % self.nc[0], (k[1] + b) % self.nc[1], (k[2] + c) % self.nc[2])
                    if q in seen:
                        continue
                    seen.add(q)
                    lst = self.cells.get(q)
                    if lst:
                        idx.extend(lst)
        return np.asarray(idx, dtype=np.int64)

    def score(self, trial_x, trial_s, idx):
        """Per trial: (all distances >= hard floor, min over atoms of r - soft target).

        trial_x [K, m, 3], trial_s [m]; idx: atoms to test against."""
        K = trial_x.shape[0]
        if self.zwall is not None:
            z = trial_x[..., 2]
            inside = np.all((z >= self.zwall[0]) & (z <= self.zwall[1]), axis=1)
        else:
            inside = np.ones(K, bool)
        if len(idx) == 0:
            return inside, np.full(K, 10.0)
        d = self.x[idx][None, None, :, :] - trial_x[:, :, None, :]
        d -= self.box * np.round(d / self.box)
        r = np.sqrt((d * d).sum(-1))                      # [K, m, n]
        hard = self.floor[trial_s[:, None], self.s[idx][None, :]]
        soft = _SOFT[trial_s[:, None], self.s[idx][None, :]]
        ok = np.all(r >= hard[None], axis=(1, 2)) & inside
        return ok, (r - soft[None]).min(axis=(1, 2))

    def add(self, p, sp, chain, pos):
        i = self.free.pop() if self.free else self.n
        if i == self.n:
            self.n += 1
        self.x[i] = p
        self.s[i] = sp
        self.chain[i] = chain
        self.pos[i] = pos
        self.alive[i] = True
        self.cells.setdefault(self._key(p), []).append(i)
        return i

    def remove(self, i):
        self.cells[self._key(self.x[i])].remove(i)
        self.alive[i] = False
        self.free.append(i)

    def compact(self):
        """Drop removed slots; order atoms chain by chain, backbone position, C before H."""
        keep = np.where(self.alive[:self.n])[0]
        order = keep[np.lexsort((self.s[keep], self.pos[keep], self.chain[keep]))]
        return self.x[order].copy(), self.s[order].copy()


def _ch2_h_batch(prev, cur, nxt):
    """CH2 hydrogens of carbon cur for a batch of next-carbon positions nxt [K,3] -> [K,2,3]."""
    a = _unit(prev - cur)
    b = nxt - cur
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    u = -(a + b)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    n = np.cross(np.broadcast_to(a, b.shape), b)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    half = TETRA / 2.0
    h1 = cur + CH * (math.cos(half) * u + math.sin(half) * n)
    h2 = cur + CH * (math.cos(half) * u - math.sin(half) * n)
    return np.stack([h1, h2], axis=1)


def _nerf_batch(a, b, c, bond, angle, tors):
    bc = _unit(c - b)
    n = _unit(np.cross(b - a, bc))
    m = np.cross(n, bc)
    return (c + (-bond * math.cos(angle)) * bc + (bond * math.sin(angle) * np.cos(tors))[:, None] * m
            + (bond * math.sin(angle) * np.sin(tors))[:, None] * n)


class _Chain:
    def __init__(self, cid):
        self.cid = cid
        self.bb = []       # backbone carbon positions
        self.cidx = []     # packer index of each backbone carbon
        self.hidx = []     # packer indices of the hydrogens of each backbone carbon
        self.fails = 0
        self.done = False


def _grow_all(pk, n_chains, nC, rng, K=24, lo=None, hi=None):
    """Grow n_chains CnH(2n+2) chains together, one backbone carbon per chain
    per sweep.  Torsions are drawn uniformly; of K trials the one that best
    clears the soft distance targets is kept (never below the hard floor).  A
    chain that cannot continue backs up two units; one that keeps failing is
    removed and started again elsewhere."""
    box = pk.box
    lo = 0.0 if lo is None else lo
    hi = box[2] if hi is None else hi
    chains = [_Chain(c) for c in range(n_chains)]

    def others(ch, p, k):
        idx = pk.near(p)
        if len(idx):
            idx = idx[~((pk.chain[idx] == ch.cid) & (pk.pos[idx] >= k - 2))]
        return idx

    def seed(ch):
        for _ in range(5000):
            c0 = rng.uniform([0, 0, lo], [box[0], box[1], hi])
            c1 = c0 + _random_rotation(rng) @ np.array([CC, 0.0, 0.0])
            ok, sc = pk.score(np.array([[c0, c1]]), np.array([0, 0]), pk.near(c0))
            if ok[0] and sc[0] > 1.0:
                ch.bb = [c0, c1]
                ch.cidx = [pk.add(c0, 0, ch.cid, 0), pk.add(c1, 0, ch.cid, 1)]
                ch.hidx = [[], []]
                return
        raise RuntimeError("could not seed a chain")

    def back(ch):
        k = len(ch.bb)
        pk.remove(ch.cidx.pop())
        ch.bb.pop()
        ch.hidx.pop()
        for h in ch.hidx[k - 2]:
            pk.remove(h)
        ch.hidx[k - 2] = []

    def restart(ch):
        for lst in ch.hidx:
            for h in lst:
                pk.remove(h)
        for c in ch.cidx:
            pk.remove(c)
        ch.fails = 0
        seed(ch)

    def step(ch):
        bb, k = ch.bb, len(ch.bb)
        if k < nC:
            if k == 2:
                a = _unit(bb[0] - bb[1])
                perp = np.cross(a, rng.normal(size=(K, 3)))
                perp /= np.linalg.norm(perp, axis=1, keepdims=True)
                cand = bb[1] + CC * (math.cos(TETRA) * a + math.sin(TETRA) * perp)
                h3 = np.stack([np.array(_ch3_hydrogens(q, bb[1], bb[0])) for q in cand])
                hs = np.concatenate([h3, _ch2_h_batch(bb[0], bb[1], cand)], axis=1)
            else:
                cand = _nerf_batch(bb[k - 3], bb[k - 2], bb[k - 1], CC, TETRA, rng.uniform(-math.pi, math.pi, K))
                hs = _ch2_h_batch(bb[k - 2], bb[k - 1], cand)
            T = np.concatenate([hs, cand[:, None, :]], axis=1)
        else:
            rot = rng.uniform(-math.pi, math.pi, K)
            T = np.array([[_nerf(bb[-3], bb[-2], bb[-1], CH, TETRA, r0 + t)
                           for t in (0.0, 2 * math.pi / 3, -2 * math.pi / 3)] for r0 in rot])
        sp = np.array([1] * (T.shape[1] - 1) + [1 if k == nC else 0])
        ok, sc = pk.score(T, sp, others(ch, bb[-1], k))
        if not ok.any():
            return False
        atoms = T[int(np.argmax(np.where(ok, sc, -1e9)))]
        if k == nC:
            ch.hidx[nC - 1] = [pk.add(h, 1, ch.cid, nC - 1) for h in atoms]
            ch.done = True
            return True
        if k == 2:
            ch.hidx[0] = [pk.add(h, 1, ch.cid, 0) for h in atoms[:3]]
            ch.hidx[1] = [pk.add(h, 1, ch.cid, 1) for h in atoms[3:5]]
        else:
            ch.hidx[k - 1] = [pk.add(h, 1, ch.cid, k - 1) for h in atoms[:2]]
        ch.cidx.append(pk.add(atoms[-1], 0, ch.cid, k))
        ch.bb.append(atoms[-1])
        ch.hidx.append([])
        return True

    for ch in chains:
        seed(ch)
    sweeps = 0
    while not all(ch.done for ch in chains):
        sweeps += 1
        if sweeps > 100 * nC:
            raise RuntimeError("chain growth did not converge")
        for c in rng.permutation(n_chains):
            ch = chains[c]
            if ch.done:
                continue
            if step(ch):
                continue
            ch.fails += 1
            if ch.fails > 25 or len(ch.bb) <= 4:
                restart(ch)
                continue
            for _ in range(min(2, len(ch.bb) - 3)):
                back(ch)


def _chain_topology(chain, pos, s):
    """Bonds and bond-angle (1-3) pairs of grown alkane chains from their labels."""
    n = len(s)
    key = {}
    hyd = {}
    for i in range(n):
        if s[i] == 0:
            key[(int(chain[i]), int(pos[i]))] = i
        else:
            hyd.setdefault((int(chain[i]), int(pos[i])), []).append(i)
    nb = [[] for _ in range(n)]
    bonds = []
    for (c, k), i in key.items():
        j = key.get((c, k + 1))
        if j is not None:
            bonds.append((i, j)); nb[i].append(j); nb[j].append(i)
        for h in hyd.get((c, k), []):
            bonds.append((i, h)); nb[i].append(h); nb[h].append(i)
    ang = set()
    for i in range(n):
        for a in range(len(nb[i])):
            for b in range(a + 1, len(nb[i])):
                p, q = sorted((nb[i][a], nb[i][b]))
                ang.add((p, q))
    return np.array(bonds, dtype=np.int64), np.array(sorted(ang), dtype=np.int64)


def _relax(x, s, box, bonds, angles, zwall=None, iters=3000, log=None):
    """Push non-bonded atoms apart while springs hold bond lengths and bond
    angles (as 1-3 distances) at their grown values: plain capped-step
    gradient descent on a quadratic penalty.  Geometry only."""
    from scipy.spatial import cKDTree
    box = np.asarray(box, float)
    x = np.mod(x, box)

    def disp(a, b):
        d = x[b] - x[a]
        return d - box * np.round(d / box)

    r0b = np.linalg.norm(disp(bonds[:, 0], bonds[:, 1]), axis=1)
    r0a = np.linalg.norm(disp(angles[:, 0], angles[:, 1]), axis=1)
    excl = set(map(tuple, bonds.tolist())) | set(map(tuple, angles.tolist()))
    excl_code = np.array(sorted(a * len(s) + b for a, b in excl), dtype=np.int64)
    hard = _HARD[s[:, None], s[None, :]] if len(s) < 2 else None
    pairs = None
    for it in range(iters):
        if it % 10 == 0:
            tree = cKDTree(np.mod(x, box), boxsize=box)
            pairs = tree.query_pairs(2.7, output_type="ndarray")
            pairs.sort(axis=1)
            code = pairs[:, 0] * len(s) + pairs[:, 1]
            pairs = pairs[~np.isin(code, excl_code)]
        g = np.zeros_like(x)
        d = disp(pairs[:, 0], pairs[:, 1])
        r = np.linalg.norm(d, axis=1)
        tgt = _RELAX[s[pairs[:, 0]], s[pairs[:, 1]]]
        viol = r < tgt
        f = np.where(viol, 20.0 * (r - tgt) / np.maximum(r, 1e-9), 0.0)[:, None] * d
        np.add.at(g, pairs[:, 0], f)
        np.add.at(g, pairs[:, 1], -f)
        for lst, r0, k in ((bonds, r0b, 4.0), (angles, r0a, 1.0)):
            d2 = disp(lst[:, 0], lst[:, 1])
            r2 = np.linalg.norm(d2, axis=1)
            f2 = (k * (r2 - r0) / r2)[:, None] * d2
            np.add.at(g, lst[:, 0], f2)
            np.add.at(g, lst[:, 1], -f2)
        step = 0.05 * g
        m = np.linalg.norm(step, axis=1)
        step *= np.minimum(1.0, 0.05 / np.maximum(m, 1e-12))[:, None]
        x = x + step
        if zwall is not None:
            x[:, 2] = np.clip(x[:, 2], zwall[0], zwall[1])
        hard_viol = (r < _HARD[s[pairs[:, 0]], s[pairs[:, 1]]]).sum()
        if log and it % 100 == 0:
            log(it, int(viol.sum()), int(hard_viol), float(r.min()) if len(r) else 0.0)
        if it % 10 == 9 and hard_viol == 0 and it >= 99:
            break
    return np.mod(x, box)


def polyethylene(n_chains, n_carbon, box, seed, T=300.0, jitter=0.0, zwall=None, relax=None, log=None):
    """n_chains CnH(2n+2) chains grown with uniform random torsions in a periodic box.

    At melt density (relax=True) the chains are grown with a low overlap floor
    and then relaxed so that every non-bonded pair clears the bonding range."""
    rng = np.random.default_rng(seed)
    per_chain = 3 * n_carbon + 2
    if relax is None:
        relax = n_chains * per_chain / float(np.prod(box)) > 0.05
    pk = _Packer(box, n_chains * per_chain + 64, zwall=zwall, floor=_GROW_FLOOR if relax else None)
    lo, hi = (zwall[0] + 1.0, zwall[1] - 1.0) if zwall is not None else (None, None)
    _grow_all(pk, n_chains, n_carbon, rng, lo=lo, hi=hi)
    meta = dict(kind="polyethylene", n_chains=n_chains, n_carbon=n_carbon, seed=seed)
    if relax:
        keep = np.where(pk.alive[:pk.n])[0]
        order = keep[np.lexsort((pk.s[keep], pk.pos[keep], pk.chain[keep]))]
        x, s_, ch, ps = pk.x[order], pk.s[order], pk.chain[order], pk.pos[order]
        bonds, angles = _chain_topology(ch, ps, s_)
        x = _relax(x, s_, box, bonds, angles, zwall=zwall, log=log)
        out = dict(x=x, species=s_.copy(), box=np.asarray(box, float), periodic=np.ones(3, np.int32), meta=meta)
        if T is not None:
            out["v"] = maxwell_velocities(s_, T, rng)
        return out
    return _finish(pk, box, (1, 1, 1), rng, T, meta, jitter)


def _finish(pk, box, periodic, rng, T, meta, jitter=0.0):
    x, s = pk.compact()
    if jitter > 0:
        x += rng.normal(scale=jitter, size=x.shape)
    for c in range(3):
        if periodic[c]:
            x[:, c] %= box[c]
    out = dict(x=x, species=s, box=np.asarray(box, float), periodic=np.asarray(periodic, np.int32), meta=meta)
    if T is not None:
        out["v"] = maxwell_velocities(s, T, rng)
    return out


DATA = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)), "data")


def cached(name, make):
    """Load a generated system from data/<name>.npz, generating and storing it if absent."""
    import os
    path = os.path.join(DATA, name + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        out = {k: z[k] for k in z.files if k != "meta_json"}
        import json
        out["meta"] = json.loads(str(z["meta_json"]))
        return out
    d = make()
    import json
    os.makedirs(DATA, exist_ok=True)
    arrs = {k: v for k, v in d.items() if k != "meta"}
    np.savez_compressed(path, meta_json=json.dumps(d["meta"]), **arrs)
    return d


def pe_small(seed=SEED0 + 0, T=300.0):
    """4 x C20H42 in a 20 A periodic cube, Gaussian jitter 0.05 A (248 atoms)."""
    return polyethylene(4, 20, (20.0, 20.0, 20.0), seed, T=T, jitter=0.05)


def melt_box_side(n_atoms_per_chain, n_chains, density_gcc=0.85):
    mass = n_chains * (n_atoms_per_chain // 3 * MASS[0] + (n_atoms_per_chain - n_atoms_per_chain // 3) * MASS[1])
    return (mass * 1.66053906660 / density_gcc) ** (1.0 / 3.0)


def pe_melt(n_chains=106, n_carbon=100, density_gcc=0.85, seed=SEED0 + 1, T=300.0, shape=(1.0, 1.0, 1.0),
            use_cache=True):
    """C100H202 melt at 0.85 g/cm^3 (106 chains = 32,012 atoms, cube 66.26 A).

    shape scales the box sides at fixed volume (for slabs that must match a
    crystal's in-plane cell)."""
    per = 3 * n_carbon + 2
    mass = n_chains * (n_carbon * MASS[0] + (2 * n_carbon + 2) * MASS[1])
    vol = mass * 1.66053906660 / density_gcc
    sh = np.asarray(shape, float)
    L = vol ** (1.0 / 3.0) * sh / np.prod(sh) ** (1.0 / 3.0)

    def make():
        out = polyethylene(n_chains, n_carbon, tuple(L), seed, T=T)
        out["meta"].update(kind="pe_melt", density_gcc=density_gcc, atoms_per_chain=per)
        return out
    if not use_cache:
        return make()
    tag = f"pe_melt_{n_chains}x{n_carbon}_s{seed}_" + "x".join(f"{v:.2f}" for v in L)
    return cached(tag, make)


def tile(sysd, reps):
    """Periodic replica reps = (a, b, c) of a periodic system."""
    x, s, box = sysd["x"], sysd["species"], np.asarray(sysd["box"])
    shifts = np.array([[a, b, c] for a in range(reps[0]) for b in range(reps[1]) for c in range(reps[2])], float)
    X = (x[None, :, :] + (shifts * box)[:, None, :]).reshape(-1, 3)
    S = np.tile(s, len(shifts))
    out = dict(x=X, species=S, box=box * np.asarray(reps), periodic=np.asarray(sysd["periodic"]),
               meta=dict(sysd["meta"], tiled=list(reps)))
    if "v" in sysd:
        out["v"] = np.tile(sysd["v"], (len(shifts), 1))
    return out


def isolated(x, species, pad=20.0):
    """A molecule in a non-periodic box (box lengths only bound the coordinates)."""
    x = np.asarray(x, float)
    lo = x.min(0)
    x = x - lo + pad / 2
    box = x.max(0) + pad / 2
    return dict(x=x, species=np.asarray(species, np.int32), box=box, periodic=np.zeros(3, np.int32),
                meta=dict(kind="isolated"))


# ---------------------------------------------------------------------------
# Small molecules (tests)
# ---------------------------------------------------------------------------
def alkane(n_carbon, torsions=None, rng=None):
    """CnH(2n+2) with given backbone torsions (radians; default all-trans)."""
    if n_carbon == 1:
        c = np.zeros(3)
        d = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / math.sqrt(3)
        return np.vstack([c, c + CH * d]), np.array([0, 1, 1, 1, 1], np.int32)
    bb = [np.zeros(3), np.array([CC, 0, 0])]
    if n_carbon > 2:
        bb.append(bb[1] + np.array([-CC * math.cos(TETRA), CC * math.sin(TETRA), 0]))
    for k in range(3, n_carbon):
        t = math.pi if torsions is None else torsions[k - 3]
        bb.append(_nerf(bb[k - 3], bb[k - 2], bb[k - 1], CC, TETRA, t))
    xs, ss = list(bb), [0] * n_carbon
    if n_carbon == 2:
        ref = np.array([0, 1.0, 0])
        for h in _ch3_hydrogens(ref + bb[1], bb[1], bb[0]):
            xs.append(h); ss.append(1)
        for h in _ch3_hydrogens(ref + bb[0], bb[0], bb[1]):
            xs.append(h); ss.append(1)
        return np.array(xs), np.array(ss, np.int32)
    for h in _ch3_hydrogens(bb[2], bb[1], bb[0]):
        xs.append(h); ss.append(1)
    for k in range(1, n_carbon - 1):
        for h in _ch2_hydrogens(bb[k - 1], bb[k], bb[k + 1]):
            xs.append(h); ss.append(1)
    for h in _ch3_hydrogens(bb[-3], bb[-2], bb[-1]):
        xs.append(h); ss.append(1)
    return np.array(xs), np.array(ss, np.int32)


def ethane(phi):
    """Ethane with the H-C-C-H dihedral set by rotating one methyl group by phi (radians)."""
    c0, c1 = np.zeros(3), np.array([CC, 0, 0])
    ref = np.array([0.0, 1.0, 0.0])
    h0 = [_nerf(ref + c1, c1, c0, CH, TETRA, t) for t in (0, 2 * math.pi / 3, -2 * math.pi / 3)]
    h1 = [_nerf(ref, c0, c1, CH, TETRA, phi + t) for t in (0, 2 * math.pi / 3, -2 * math.pi / 3)]
    return np.vstack([c0, c1] + h0 + h1), np.array([0, 0, 1, 1, 1, 1, 1, 1], np.int32)


def ring_aromatic(n_rings=1, cc=1.40):
    """Benzene (1), naphthalene (2), anthracene (3): planar, C-H 1.09 A."""
    centres = [np.array([k * cc * math.sqrt(3), 0.0, 0.0]) for k in range(n_rings)]
    pts = []
    for c in centres:
        for m in range(6):
            a = math.pi / 6 + m * math.pi / 3
            p = c + cc * np.array([math.cos(a), math.sin(a), 0.0])
            if not any(np.linalg.norm(p - q) < 0.1 for q in pts):
                pts.append(p)
    C = np.array(pts)
    xs, ss = [*C], [0] * len(C)
    for i, p in enumerate(C):
        nb = [q for q in C if 0.1 < np.linalg.norm(q - p) < cc * 1.1]
        if len(nb) == 2:
            d = _unit(2 * p - nb[0] - nb[1])
            xs.append(p + CH * d); ss.append(1)
    return np.array(xs), np.array(ss, np.int32)


def ethylene(cc=1.33):
    """Planar C2H4 with exact 120 degree angles."""
    c0, c1 = np.zeros(3), np.array([cc, 0, 0])
    hs = []
    for c, sgn in ((c0, -1), (c1, 1)):
        for a in (math.pi / 3, -math.pi / 3):
            hs.append(c + CH * np.array([sgn * math.cos(a), math.sin(a), 0.0]))
    return np.vstack([c0, c1] + hs), np.array([0, 0, 1, 1, 1, 1], np.int32)


def graphene_flake(nx, ny, cc=1.42):
    """Parallelogram of nx x ny fused hexagons (a polycyclic aromatic
    hydrocarbon; 2 x 2 is pyrene C16H10), H on every two-fold carbon.

    Built as the union of the rings' vertices, so every carbon lies on a
    ring and has two or three carbon neighbours: no bare chain ends."""
    a = cc * math.sqrt(3)
    A1 = np.array([a, 0.0, 0.0])
    A2 = np.array([a / 2, 1.5 * cc, 0.0])
    pts = []
    for i in range(nx):
        for j in range(ny):
            c = i * A1 + j * A2
            for m in range(6):
                t = math.pi / 6 + m * math.pi / 3
                p = c + cc * np.array([math.cos(t), math.sin(t), 0.0])
                if not any(np.linalg.norm(p - q) < 0.1 for q in pts):
                    pts.append(p)
    C = np.array(pts)
    d = np.linalg.norm(C[:, None] - C[None], axis=2)
    xs, ss = [*C], [0] * len(C)
    for i in range(len(C)):
        nb = np.where((d[i] > 0.1) & (d[i] < cc * 1.1))[0]
        if len(nb) == 2:
            v = _unit(2 * C[i] - C[nb[0]] - C[nb[1]])
            xs.append(C[i] + CH * v); ss.append(1)
    return np.array(xs), np.array(ss, np.int32)


def nanotube(n, m, ncells, cc=1.42):
    """Single-wall (n, m) carbon nanotube along z, ncells translational unit
    cells long, periodic along its axis.

    The graphene sheet (lattice constant a = sqrt(3) cc) is rolled so that
    the chiral vector C = n a1 + m a2 becomes the circumference and the
    translation vector T (the shortest lattice vector normal to C) the axis.
    Returns (x [N, 3], species (all carbon), box, periodic) with the tube
    centred in a box whose x and y sides leave 20 A of vacuum and are not
    periodic, and whose z side is ncells |T|."""
    a = cc * math.sqrt(3.0)
    a1 = np.array([a * math.sqrt(3.0) / 2, a / 2])
    a2 = np.array([a * math.sqrt(3.0) / 2, -a / 2])
    basis = [np.zeros(2), (a1 + a2) / 3.0]
    dr = math.gcd(2 * m + n, 2 * n + m)
    t1, t2 = (2 * m + n) // dr, -(2 * n + m) // dr
    C = n * a1 + m * a2
    T = t1 * a1 + t2 * a2
    Lc, Lt = float(np.linalg.norm(C)), float(np.linalg.norm(T))
    per_cell = 4 * (n * n + n * m + m * m) // dr
    pts = []
    span = n + m + abs(t1) + abs(t2) + 2
    for i in range(-span, span + 1):
        for j in range(-span, span + 1):
            for b in basis:
                p = i * a1 + j * a2 + b
                u = float(p @ C) / Lc ** 2          # fraction of the circumference
                w = float(p @ T) / Lt ** 2          # fraction of the cell length
                if -1e-9 <= u < 1 - 1e-9 and -1e-9 <= w < 1 - 1e-9:
                    pts.append((u, w))
    if len(pts) != per_cell:
        raise RuntimeError(f"({n},{m}) unit cell: {len(pts)} atoms, expected {per_cell}")
    R = Lc / (2 * math.pi)
    L = ncells * Lt
    side = 2 * R + 40.0
    xs = []
    for k in range(ncells):
        for u, w in pts:
            th = 2 * math.pi * u
            xs.append([side / 2 + R * math.cos(th), side / 2 + R * math.sin(th), (w + k) * Lt])
    x = np.array(xs)
    return x, np.zeros(len(x), np.int32), np.array([side, side, L]), np.array([0, 0, 1], np.int32)


def nanotube_bundle(n=10, m=10, ncells=40, nx=4, ny=4, gap=3.4, seed=SEED0 + 5, T=300.0):
    """nx x ny parallel (n, m) nanotubes on a square lattice, gap A between
    walls, in a box periodic in all three directions (the tubes infinite
    along z); Maxwell velocities at T.  The default is 16 (10,10) tubes of
    40 cells: 25,600 carbon atoms, 67.8 x 67.8 x 98.4 A."""
    x0, s0, box0, _ = nanotube(n, m, ncells)
    c0 = np.array([box0[0] / 2, box0[1] / 2, 0.0])
    rad = float(np.linalg.norm(x0[0, :2] - c0[:2]))
    pitch = 2 * rad + gap
    xs = []
    for i in range(nx):
        for j in range(ny):
            xs.append(x0 - c0 + np.array([(i + 0.5) * pitch, (j + 0.5) * pitch, 0.0]))
    x = np.vstack(xs)
    s = np.zeros(len(x), np.int32)
    box = np.array([nx * pitch, ny * pitch, box0[2]])
    v = maxwell_velocities(s, T, np.random.default_rng(seed))
    return dict(x=x, species=s, v=v, box=box, periodic=np.ones(3, np.int32),
                meta=dict(kind="nanotube_bundle", n=n, m=m, ncells=ncells, nx=nx, ny=ny, seed=seed))


# ---------------------------------------------------------------------------
# Crystalline slabs and the ~10^6-atom hybrid system
# ---------------------------------------------------------------------------
DIAMOND_A = 3.567
GRAPHITE_CC = 1.42
GRAPHITE_GAP = 3.35


def graphite_stack(nx, ny, layers, lx=None, ly=None):
    """AB graphite: nx x ny rectangular cells (a, 3 d) of 4 atoms per layer,
    optionally scaled in-plane to lx, ly; layers 3.35 A apart, origin at z = 0."""
    d = GRAPHITE_CC
    a = d * math.sqrt(3.0)
    basis = np.array([[0, 0], [a / 2, d / 2], [a / 2, 1.5 * d], [0, 2 * d]])
    cells = np.array([[i * a, j * 3 * d] for i in range(nx) for j in range(ny)])
    layer = (cells[:, None, :] + basis[None]).reshape(-1, 2)
    sx = 1.0 if lx is None else lx / (nx * a)
    sy = 1.0 if ly is None else ly / (ny * 3 * d)
    out = []
    for k in range(layers):
        xy = layer + (np.array([0.0, d]) if k % 2 else 0.0)
        z = np.full((len(xy), 1), k * GRAPHITE_GAP)
        out.append(np.hstack([xy * [sx, sy], z]))
    x = np.vstack(out)
    x[:, 1] %= ny * 3 * d * sy
    return x, np.zeros(len(x), np.int32)


def diamond111_slab(nx, ny, bilayers, a=DIAMOND_A, lx=None, ly=None):
    """H-terminated diamond (111) slab: orthorhombic cells (a/sqrt2, a sqrt6/2)
    in-plane, `bilayers` (111) bilayers, one H per dangling bond, origin z = 0."""
    R = np.array([[1, -1, 0], [1, 1, -2], [1, 1, 1]], float)
    R /= np.linalg.norm(R, axis=1, keepdims=True)
    c1, c2, c3 = a / math.sqrt(2), a * math.sqrt(6) / 2, a * math.sqrt(3)
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    basis = np.vstack([fcc, fcc + 0.25]) * a
    rng_ = range(-4, 5)
    pts = np.array([[i, j, k] for i in rng_ for j in rng_ for k in rng_], float) * a
    lat = (pts[:, None, :] + basis[None]).reshape(-1, 3) @ R.T
    frac = lat / [c1, c2, c3]
    keep = np.all((frac >= -1e-6) & (frac < 1 - 1e-6), axis=1)
    cell = lat[keep]
    assert len(cell) == 12, len(cell)
    nz = bilayers // 3 + 2
    reps = np.array([[i, j, k] for i in range(nx) for j in range(ny) for k in range(nz)], float) * [c1, c2, c3]
    C = (reps[:, None, :] + cell[None]).reshape(-1, 3)
    # bilayers: z-levels come in pairs 0.515 A apart; cut through the 1.545 A vertical bonds
    zs = np.unique(np.round(C[:, 2], 3))
    pairs = [(zs[i], zs[i + 1]) for i in range(0, len(zs) - 1) if zs[i + 1] - zs[i] < 0.8]
    # choose pairs that form true bilayers (first of each pair is the lower sublayer)
    bl = []
    for lo, hi in pairs:
        if not bl or lo > bl[-1][1] + 0.1:
            bl.append((lo, hi))
    bl = bl[1:1 + bilayers]
    zmin, zmax = bl[0][0] - 0.01, bl[-1][1] + 0.01
    C = C[(C[:, 2] >= zmin) & (C[:, 2] <= zmax)]
    C[:, 2] -= C[:, 2].min()
    L = np.array([nx * c1, ny * c2])
    # hydrogens on under-coordinated surface carbons
    from scipy.spatial import cKDTree
    xy = C.copy()
    xy[:, :2] %= L
    xy[:, :2] = np.where(xy[:, :2] >= L, xy[:, :2] - L, xy[:, :2])
    tree = cKDTree(xy, boxsize=[L[0], L[1], 1e6])
    pairs = tree.query_pairs(1.7, output_type="ndarray")
    deg = np.bincount(pairs.ravel(), minlength=len(C))
    nbsum = np.zeros_like(C)
    for a_, b_ in ((0, 1), (1, 0)):
        d = xy[pairs[:, b_]] - xy[pairs[:, a_]]
        d[:, :2] -= L * np.round(d[:, :2] / L)
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        np.add.at(nbsum, pairs[:, a_], d)
    H = []
    for i in np.where(deg == 3)[0]:
        u = -nbsum[i] / np.linalg.norm(nbsum[i])
        H.append(xy[i] + CH * u)
    x = np.vstack([xy, np.array(H)])
    s = np.concatenate([np.zeros(len(xy), np.int32), np.ones(len(H), np.int32)])
    if lx is not None:
        sc = np.array([lx / L[0], ly / L[1]])
        x[:, :2] = (x[:, :2] % L) * sc
        L = L * sc
    return x, s, L


def pe_melt_cell(n_chains, lx, ly, density_gcc=0.85, n_carbon=100, seed=SEED0 + 21, T=300.0):
    """Periodic melt cell with in-plane sides lx, ly (cached like pe_melt)."""
    mass = n_chains * (n_carbon * MASS[0] + (2 * n_carbon + 2) * MASS[1])
    lz = mass * 1.66053906660 / density_gcc / (lx * ly)
    return pe_melt(n_chains, n_carbon, density_gcc, seed, T, shape=(lx, ly, lz))


def hybrid_1m(seed=SEED0 + 2, T=300.0, melt_tiles=(2, 2, 5)):
    """~10^6 atoms: AB graphite stack (30 layers), H-terminated diamond (111)
    slab (31 bilayers) and a polyethylene melt slab (tiles of the 32,012-atom
    melt), stacked along z with 3.4 A gaps in one periodic box.  The in-plane
    cell is that of the tiled melt; the crystals are strained to it (diamond
    by about 1%, graphite by about 0.3%)."""
    tile = pe_melt()
    tb = tile["box"]
    lx, ly = melt_tiles[0] * tb[0], melt_tiles[1] * tb[1]
    c1, c2 = DIAMOND_A / math.sqrt(2), DIAMOND_A * math.sqrt(6) / 2
    dx, ds, L = diamond111_slab(int(round(lx / c1)), int(round(ly / c2)), 31, lx=lx, ly=ly)
    ga = GRAPHITE_CC * math.sqrt(3)
    gx, gs = graphite_stack(int(round(lx / ga)), int(round(ly / (3 * GRAPHITE_CC))), 30, lx=lx, ly=ly)
    # unwrap every chain of the melt cell along z (atoms of a chain are stored
    # together; each atom taken at the image nearest to the previous one)
    per = 3 * 100 + 2
    cz = tile["x"][:, 2].reshape(-1, per).copy()
    step = np.diff(cz, axis=1)
    cz[:, 1:] = cz[:, :1] + np.cumsum(step - tb[2] * np.round(step / tb[2]), axis=1)
    cell = tile["x"].copy()
    cell[:, 2] = cz.ravel()
    reps = [(a, b, c) for a in range(melt_tiles[0]) for b in range(melt_tiles[1]) for c in range(melt_tiles[2])]
    mx = np.vstack([cell + np.array(r) * tb for r in reps])
    ms = np.tile(tile["species"], len(reps))
    # stacked copies stay continuous inside the block; chains that cross the
    # block's outer z faces (which border the crystals) are removed whole
    hz = melt_tiles[2] * tb[2]
    nch = len(ms) // per
    zc = mx[:, 2].reshape(nch, per)
    keep = (zc.min(1) >= 0.0) & (zc.max(1) < hz)
    mx = mx.reshape(nch, per, 3)[keep].reshape(-1, 3)
    ms = ms.reshape(nch, per)[keep].ravel()
    mx[:, :2] %= [melt_tiles[0] * tb[0], melt_tiles[1] * tb[1]]
    gap = 3.4
    parts, z = [], 0.0
    for x, s in ((gx, gs), (dx, ds), (mx, ms)):
        x = x.copy()
        x[:, 2] += z - x[:, 2].min()
        parts.append((x, s))
        z = x[:, 2].max() + gap
    X = np.vstack([p[0] for p in parts])
    S = np.concatenate([p[1] for p in parts])
    box = np.array([lx, ly, z])
    X[:, :2] %= box[:2]
    rng = np.random.default_rng(seed)
    V = maxwell_velocities(S, T, rng)
    meta = dict(kind="hybrid_1m", graphite=len(gs), diamond=int((ds == 0).sum()), diamond_h=int((ds == 1).sum()),
                melt=len(ms), melt_chains=int(keep.sum()), seed=seed)
    return dict(x=X, species=S, box=box, periodic=np.ones(3, np.int32), v=V, meta=meta)


# ---------------------------------------------------------------------------
# Batches of small systems
# ---------------------------------------------------------------------------
def diamond_cluster(radius, a=DIAMOND_A):
    """H-terminated piece of diamond: lattice sites within `radius` of the
    origin, every missing tetrahedral bond capped with H (carbons left with
    no carbon neighbour are dropped)."""
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    n = int(math.ceil(radius / a)) + 1
    cells = np.array([[i, j, k] for i in range(-n, n + 1) for j in range(-n, n + 1) for k in range(-n, n + 1)], float)
    A = ((cells[:, None] + fcc[None]) * a).reshape(-1, 3)
    B = A + a / 4
    dirs_a = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / 4 * a
    sites = [(p, +1) for p in A if np.linalg.norm(p) <= radius] + [(p, -1) for p in B if np.linalg.norm(p) <= radius]
    pos = np.array([p for p, _ in sites])
    sub = np.array([g for _, g in sites])
    key = {tuple(np.round(p, 3)): i for i, p in enumerate(pos)}
    # grow the site set until no empty site has two or more occupied neighbours
    # (two caps pointing into one vacancy would collide)
    changed = True
    while changed:
        changed = False
        cand = {}
        for p, g in zip(pos, sub):
            for d in dirs_a:
                q = tuple(np.round(p + g * d, 3))
                if q not in key:
                    cand.setdefault(q, [np.array(q), -g, 0])[2] += 1
        for q, (p, g, cnt) in cand.items():
            if cnt >= 2:
                key[q] = len(pos)
                pos = np.vstack([pos, p])
                sub = np.append(sub, g)
                changed = True
    keep = []
    for i, (p, g) in enumerate(zip(pos, sub)):
        nbc = sum(tuple(np.round(p + g * d, 3)) in key for d in dirs_a)
        if nbc >= 1:
            keep.append(i)
    keepset = set(keep)
    xs, ss = [], []
    for i in keep:
        xs.append(pos[i]); ss.append(0)
        for d in dirs_a:
            q = tuple(np.round(pos[i] + sub[i] * d, 3))
            if q not in key or key[q] not in keepset:
                xs.append(pos[i] + sub[i] * d / np.linalg.norm(d) * CH); ss.append(1)
    return np.array(xs), np.array(ss, np.int32)


def branched_alkane(n_carbon, rng):
    """Alkane backbone with one or two methyl branches replacing hydrogens."""
    x, s = alkane(n_carbon, torsions=list(rng.choice([math.pi, math.pi / 3, -math.pi / 3], size=max(0, n_carbon - 3))))
    hs = np.where(s == 1)[0]
    for h in rng.choice(hs, size=min(2, len(hs)), replace=False):
        # carbon bonded to this hydrogen
        c = int(np.argmin(np.where(s == 0, np.linalg.norm(x - x[h], axis=1), 1e9)))
        u = _unit(x[h] - x[c])
        cnew = x[c] + CC * u
        ref = x[c] + np.cross(u, rng.normal(size=3))
        hs3 = [_nerf(ref, x[c], cnew, CH, TETRA, t) for t in (0, 2 * math.pi / 3, -2 * math.pi / 3)]
        x = np.vstack([x[:h], [cnew], x[h + 1:], hs3])
        s = np.concatenate([s[:h], [0], s[h + 1:], [1, 1, 1]]).astype(np.int32)
    return x, s


FAMILIES = ("linear_alkane", "branched_alkane", "aromatic", "graphene_flake", "diamond_cluster")


def _clean(x, s):
    """True when every pair closer than the REBO range is a proper bond
    (C-C 1.3-1.6 A, C-H 1.0-1.15 A, no H-H pair below 1.7 A) and every
    atom is saturated: each H has one bonded neighbour and each C three
    (sp2) or four (sp3).  A bare carbon is a radical that reacts in the
    first picoseconds of dynamics."""
    d = np.linalg.norm(x[:, None] - x[None], axis=2)
    iu = np.triu_indices(len(s), 1)
    dd, a, b = d[iu], s[iu[0]], s[iu[1]]
    hh = (a == 1) & (b == 1)
    ch = (a + b) == 1
    cc = (a == 0) & (b == 0)
    bad = (hh & (dd < 1.7)) | (ch & ((dd < 1.0) | ((dd > 1.15) & (dd < 1.8)))) | \
          (cc & ((dd < 1.3) | ((dd > 1.6) & (dd < 2.0))))
    if bad.any():
        return False
    sa, sb = s[:, None], s[None, :]
    bonded = np.where((sa == 0) & (sb == 0), d < 1.6, np.where(sa + sb == 1, d < 1.15, False))
    np.fill_diagonal(bonded, False)
    deg = bonded.sum(1)
    return bool(np.all(deg[s == 1] == 1) and np.all((deg[s == 0] >= 3) & (deg[s == 0] <= 4)))


def molecule(family, rng, tries=400):
    """A random molecule of the family whose geometry is chemically clean."""
    for _ in range(tries):
        x, s = _molecule(family, rng)
        if _clean(x, s):
            return x, s
    raise RuntimeError(f"could not build a clean {family} molecule")


def _molecule(family, rng):
    if family == "linear_alkane":
        k = int(rng.integers(4, 17))
        return alkane(k, torsions=list(rng.choice([math.pi, math.pi / 3, -math.pi / 3], size=max(0, k - 3))))
    if family == "branched_alkane":
        return branched_alkane(int(rng.integers(5, 13)), rng)
    if family == "aromatic":
        return ring_aromatic(int(rng.integers(1, 4)))
    if family == "graphene_flake":
        return graphene_flake(int(rng.integers(2, 5)), int(rng.integers(2, 4)))
    return diamond_cluster(float(rng.uniform(2.5, 3.8)))


def molecular_box(family, n_target, rng, density=0.02, min_side=13.0, min_dist=2.6, tries=400, image_gap=4.0,
                  n_max=None):
    """Molecules of one family at random positions and orientations in a
    periodic cube of side max((n/density)^(1/3), min_side, d + image_gap)
    until at least n_target atoms (at most max(1.1 n_target, n_target + 120),
    and n_max), d being
    the first molecule's diameter.  A molecule is placed at fresh random
    positions and orientations until no atom comes within min_dist of an
    atom already placed (bounding spheres first, atoms of the molecules
    whose spheres overlap next); placement stops after `tries` failures in a
    row.  Later molecules wider than side - image_gap are rejected, so that
    no molecule can reach its own periodic image whatever its orientation."""
    L = max((n_target / density) ** (1.0 / 3.0), min_side)
    box = np.array([L, L, L])
    X = np.zeros((0, 3))
    S = np.zeros(0, np.int32)
    cen, rad, rng_of = [], [], []   # placed molecules: centre, bounding radius, atom range
    cap = max(1.1 * n_target, n_target + 120)   # room for one more molecule of any family
    if n_max is not None:
        cap = min(cap, n_max)
    fails = 0
    mol = None
    while len(S) < n_target and fails < tries:
        if mol is None:
            x, s = molecule(family, rng)
            if len(S) + len(s) > cap and len(S) > 0:
                fails += 1
                continue
            x = x - x.mean(0)
            diam = math.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1).max())
            if diam > L - image_gap:
                if len(S) > 0:
                    fails += 1
                    continue
                L = diam + image_gap
                box = np.array([L, L, L])
            mol = (x, s, math.sqrt((x * x).sum(1).max()))
        x0, s0, r0 = mol
        c = rng.uniform(0, L, 3)
        x = x0 @ _random_rotation(rng).T + c
        if cen:
            dc = c - np.array(cen)
            dc -= box * np.round(dc / box)
            near = np.where(np.sqrt((dc * dc).sum(1)) < r0 + np.array(rad) + min_dist)[0]
            if len(near):
                idx = np.concatenate([np.arange(*rng_of[k]) for k in near])
                d = x[:, None, :] - X[idx][None, :, :]
                d -= box * np.round(d / box)
                if (d * d).sum(-1).min() < min_dist ** 2:
                    fails += 1
                    continue
        rng_of.append((len(S), len(S) + len(s0)))
        cen.append(c)
        rad.append(r0)
        X = np.vstack([X, x])
        S = np.concatenate([S, s0])
        mol = None
        fails = 0
    return X % box, S, box


def batch_systems(nsys=512, nmin=50, nmax=5000, seed=SEED0 + 3, T=300.0):
    """nsys independent systems (sizes log-uniform in [nmin, nmax]), families
    round-robin, each in its own periodic cube; concatenated."""
    rng = np.random.default_rng(seed)
    xs, ss, vs, boxes, sizes, fams = [], [], [], [], [], []
    for k in range(nsys):
        fam = FAMILIES[k % len(FAMILIES)]
        n_target = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        x, s, box = molecular_box(fam, n_target, rng, n_max=nmax)
        xs.append(x); ss.append(s); boxes.append(box); sizes.append(len(s)); fams.append(fam)
        vs.append(maxwell_velocities(s, T, rng))
    return dict(x=np.vstack(xs), species=np.concatenate(ss), v=np.vstack(vs), boxes=np.array(boxes),
                sizes=np.array(sizes), periodic=np.ones((nsys, 3), np.int32),
                meta=dict(kind="batch", nsys=nsys, families=fams, seed=seed))


def batch_cached(nsys=512, seed=SEED0 + 3):
    def make():
        d = batch_systems(nsys, seed=seed)
        d["meta"] = {k: v for k, v in d["meta"].items() if k != "families"}
        return d
    return cached(f"batch_{nsys}_s{seed}_r4", make)   # r4: placement until the target size


# ---- seeded initial weights of the surrogate networks (training inputs) ----
# One network: W1 [64][112], b1 [64], W2 [64][64], b2, W3 [64][64], b3, w4 [64], b4 [1].
NN_LAYOUT = (("W1", (64, 112)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 64)), ("b3", (64,)),
             ("w4", (64,)), ("b4", (1,)))
NN_NPAR = sum(int(np.prod(s)) for _, s in NN_LAYOUT)


def nn_init_weights(nmodels, seed):
    """LeCun-normal weight matrices (std 1/sqrt(fan in)) and zero biases for
    each ensemble member and centre species: float32 [nmodels][2][15617]."""
    rng = np.random.default_rng(seed)
    out = np.zeros((nmodels, 2, NN_NPAR), np.float32)
    for m in range(nmodels):
        for sp in range(2):
            off = 0
            for name, shape in NN_LAYOUT:
                k = int(np.prod(shape))
                if name[0] in "Ww":
                    out[m, sp, off:off + k] = rng.normal(0.0, 1.0 / math.sqrt(shape[-1]), k)
                off += k
    return out

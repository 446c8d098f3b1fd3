"""Reference (numpy) of the library's point ordering and row schedule, for
tests that need the tiles of the block preconditioner.

The library sorts the points by grid cell (side >= the core radius times
1 + 1e-9, x fastest, stable), then orders the sorted points along the Morton
curve of their coordinates quantised to 2^b - 1 steps per axis over the
bounding box (b = min(16, 62 // dim), stable).  The block preconditioner's
tiles are 16 consecutive points of that order."""
import numpy as np


def schedule_rows(x, r_cell):
    """Caller row indices in schedule order."""
    x = np.asarray(x, dtype=np.float64)
    n, d = x.shape
    lo, hi = x.min(axis=0), x.max(axis=0)
    ext = hi - lo
    side = r_cell * (1.0 + 1e-9)
    G = np.minimum(np.maximum(1.0, np.floor(ext / side)), 1e6)
    cap = max(1024.0, 2.0 * n)
    while np.prod(G) > cap:
        k = int(np.argmax(G))
        G[k] = max(1.0, np.floor(G[k] / 2.0))
    inv = np.where(ext > 0, G / np.where(ext > 0, ext, 1.0), 0.0)
    t = (x - lo) * inv
    c = t.astype(np.int64)
    c[t < 0] = 0
    c = np.minimum(c, G.astype(np.int64) - 1)
    key = np.zeros(n, dtype=np.int64)
    for k in range(d - 1, -1, -1):
        key = key * int(G[k]) + c[:, k]
    perm = np.argsort(key, kind="stable")
    xs = x[perm]
    bits = min(16, 62 // d)
    top = float((1 << bits) - 1)
    scale = np.where(ext > 0, top / np.where(ext > 0, ext, 1.0), 0.0)
    q = np.minimum(np.maximum((xs - lo) * scale, 0.0), top).astype(np.uint64)
    mk = np.zeros(n, dtype=np.uint64)
    for k in range(d):
        v = q[:, k]
        spread = np.zeros(n, dtype=np.uint64)
        for b in range(bits):
            spread |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * d)
        mk |= spread << np.uint64(k)
    sched = np.argsort(mk, kind="stable")
    return perm[sched]


def schedule_tiles(x, r_cell, tile: int = 16):
    rows = schedule_rows(x, r_cell)
    return [rows[i:i + tile] for i in range(0, len(rows), tile)]

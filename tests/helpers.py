"""Small numpy helpers shared by the tests (independent of the library and of the oracle)."""
import numpy as np


def surviving_prim_pairs(b, pa, pb, screen):
    """Primitive pairs per shell pair that pass exp(-mu |A-B|^2) > screen, mu = ab/(a+b)."""
    pa, pb = np.asarray(pa), np.asarray(pb)
    ka, kb = b.nprim[pa].astype(np.int64), b.nprim[pb].astype(np.int64)
    cnt = ka * kb
    if not screen > 0:
        return cnt
    rep = np.repeat(np.arange(len(pa)), cnt)
    local = np.arange(int(cnt.sum())) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ea = b.expo[b.prim_off[pa][rep] + local // kb[rep]]
    eb = b.expo[b.prim_off[pb][rep] + local % kb[rep]]
    R2 = np.sum((b.center[pa] - b.center[pb]) ** 2, axis=1)[rep]
    return np.bincount(rep, weights=np.exp(-R2 * ea * eb / (ea + eb)) > screen, minlength=len(pa)).astype(np.int64)

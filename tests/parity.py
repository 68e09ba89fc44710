"""Error measures shared by the GPU parity tests.

rel       relative L2 over the flattened vector (the metric of Table 1,
          Sec. 3.1.2), in FP64 on the host.
tile_err  the same, per block of 16 consecutive points: the largest, over
          blocks, of ||got_t - ref_t|| / max(||ref_t||, rms block norm).  The
          kernels process points in 16-point tiles, so a tile that is wrong,
          dropped or duplicated has an error of order one here, while it moves
          the whole-vector figure by only about 1/sqrt(number of tiles).  The
          floor (the root-mean-square norm of a block) keeps blocks whose
          reference happens to be tiny from dominating.
"""
import numpy as np

TILE = 16


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cosine(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def tile_err(got, ref, tile=TILE):
    """Largest per-tile relative error; points on the last axis.  Arrays with
    a channel axis (d_out, C, N) are measured channel by channel (channels
    differ in scale) and the largest is returned."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    if ref.ndim == 3:
        return max(tile_err(got[:, c, :], ref[:, c, :], tile) for c in range(ref.shape[1]))
    g = got.reshape(-1, ref.shape[-1])
    r = ref.reshape(-1, ref.shape[-1])
    N = r.shape[1]
    n_t = (N + tile - 1) // tile
    pad = n_t * tile - N
    if pad:
        g = np.pad(g, ((0, 0), (0, pad)))
        r = np.pad(r, ((0, 0), (0, pad)))
    d = np.sqrt(((g - r) ** 2).reshape(g.shape[0], n_t, tile).sum(axis=(0, 2)))
    nr = np.sqrt((r ** 2).reshape(r.shape[0], n_t, tile).sum(axis=(0, 2)))
    floor = max(float(np.sqrt(np.mean(nr ** 2))), 1e-300)
    return float(np.max(d / np.maximum(nr, floor)))


def flat(grads):
    """[(dW, db), ...] device tensors -> one FP64 vector (W then b per layer)."""
    return np.concatenate([np.concatenate([dW.detach().double().cpu().numpy().ravel(),
                                           db.detach().double().cpu().numpy().ravel()]) for dW, db in grads])

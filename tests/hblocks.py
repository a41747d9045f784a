"""Writer of H-matrix block files (the format hlu_import_blocks reads,
declared in include/hlu.h), for the oracle's assembled H-matrices.

Test infrastructure: serialises an oracle HMatrix (dense blocks and the
U, V factors of low-rank blocks, cluster order) so that the device path can
factor the very same A_H."""
import numpy as np

import oracle as O


def write_blocks(H, path, blocks=None, perm=None, magic=b"HLUBLK01"):
    """Write H's leaf blocks (or the given list of them) to `path`."""
    blocks = list(O.leaves_of(H.block)) if blocks is None else list(blocks)
    perm = H.perm if perm is None else perm
    with open(path, "wb") as fh:
        fh.write(magic)
        np.array([H.n, len(blocks)], dtype="<i8").tofile(fh)
        np.asarray(perm, dtype="<i8").tofile(fh)
        for b in blocks:
            if b.kind == "F":
                hdr = [b.t.off, b.s.off, b.t.size, b.s.size, 0, 0]
                np.array(hdr, dtype="<i8").tofile(fh)
                np.asfortranarray(b.F, dtype="<f8").ravel(order="F").tofile(fh)
            else:
                k = b.U.shape[1]
                hdr = [b.t.off, b.s.off, b.t.size, b.s.size, 1, k]
                np.array(hdr, dtype="<i8").tofile(fh)
                np.asarray(b.U, dtype="<f8").ravel(order="F").tofile(fh)
                np.asarray(b.V, dtype="<f8").ravel(order="F").tofile(fh)


def read_blocks(path):
    """(perm, blocks) of a block file; each block is a dict with r0, c0, m,
    n, kind (0 dense, 1 low-rank) and F or U, V (FP64, column-major)."""
    with open(path, "rb") as fh:
        data = fh.read()
    assert data[:8] == b"HLUBLK01"
    off = 8
    n, nb = np.frombuffer(data, "<i8", 2, off)
    off += 16
    perm = np.frombuffer(data, "<i8", int(n), off).copy()
    off += 8 * int(n)
    blocks = []
    for _ in range(int(nb)):
        r0, c0, m, nc, kind, k = (int(v) for v in np.frombuffer(data, "<i8", 6, off))
        off += 48
        b = dict(r0=r0, c0=c0, m=m, n=nc, kind=kind, k=k)
        if kind == 0:
            b["F"] = np.frombuffer(data, "<f8", m * nc, off).reshape((m, nc), order="F").copy()
            off += 8 * m * nc
        else:
            b["U"] = np.frombuffer(data, "<f8", m * k, off).reshape((m, k), order="F").copy()
            off += 8 * m * k
            b["V"] = np.frombuffer(data, "<f8", nc * k, off).reshape((nc, k), order="F").copy()
            off += 8 * nc * k
        blocks.append(b)
    assert off == len(data)
    return perm, blocks


def to_dense(n, blocks):
    """The H-matrix of a block list, expanded (cluster order)."""
    A = np.zeros((n, n))
    for b in blocks:
        sl = (slice(b["r0"], b["r0"] + b["m"]), slice(b["c0"], b["c0"] + b["n"]))
        A[sl] = b["F"] if b["kind"] == 0 else b["U"] @ b["V"].T
    return A

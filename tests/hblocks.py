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

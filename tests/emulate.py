"""CPU emulation of the GPU scan's decomposition on exported tables.

Walks the dense table exported by ac_debug_export the way the kernels do:
every chunk of C symbols starts at the root ``warm`` symbols before its
first position (or at the text start) and reports the output sets of the
states it enters at its own positions.  Used only by the CPU tests, to check
the host automaton compiler and the chunking rule without a GPU."""
import numpy as np


def emulate_scan(delta, out_off, out_ids, first_output, text, chunk, warm):
    n = len(text)
    if n == 0:
        return np.zeros(0, dtype=np.uint64)
    nch = (n + chunk - 1) // chunk
    starts = np.arange(nch, dtype=np.int64) * chunk
    s = np.zeros(nch, dtype=np.int64)
    keys = []
    for t in range(-warm, chunk):
        pos = starts + t
        live = (pos >= 0) & (pos < n)
        sym = text[np.clip(pos, 0, n - 1)]
        s = np.where(live, delta[s, sym], s)
        if t < 0:
            continue
        hit = live & (s >= first_output)
        for c in np.flatnonzero(hit):
            o = int(s[c]) - first_output
            ids = out_ids[out_off[o]:out_off[o + 1]]
            e = np.uint64(pos[c])
            keys.append((e << np.uint64(32)) | ids.astype(np.uint64))
    if not keys:
        return np.zeros(0, dtype=np.uint64)
    return np.sort(np.concatenate(keys))

"""Edge lists as text, in the paper's record format ("u v s" per line, s = 1
for a positive and 0 for a negative edge; Section III).

Formatting only: no counting arithmetic.  Raw ids are the graph's compact ids
sent through an injective map into a wide id space, so that reading the text
back must compact them again.  ``edge_text`` writes fixed-width fields with
NumPy (fast enough for 50 M lines); ``messy_edge_text`` writes a small text
in Python with every variation the reader accepts (separators, sign
conventions, comments, blank lines, CRLF, leading zeros, no final newline).
"""

from __future__ import annotations

import numpy as np

# odd multipliers: x -> x * a mod 2^40 is a bijection on [0, 2^40)
_MUL = (0x9E3779B97, 0xC2B2AE3D27)
_MASK = (1 << 40) - 1


def raw_ids(n: int, side: int) -> np.ndarray:
    """The raw id of compact id 0 .. n - 1 of one side (distinct, < 2^40)."""
    x = np.arange(n, dtype=np.uint64)
    return ((x * np.uint64(_MUL[side])) & np.uint64(_MASK)).astype(np.int64)


def _digits(x: np.ndarray, width: int) -> np.ndarray:
    """[len(x), width] ASCII digits of x, zero-padded."""
    out = np.empty((x.shape[0], width), np.uint8)
    y = x.astype(np.uint64)
    for k in range(width - 1, -1, -1):
        out[:, k] = (y % np.uint64(10)).astype(np.uint8) + ord("0")
        y //= np.uint64(10)
    return out


def edge_text(n_u: int, n_v: int, u, v, sign, remap: bool = True) -> bytes:
    """One line per record: "<u> <v> <s>\\n", ids zero-padded to a fixed
    width (13 digits with ``remap``, else the width of the largest id)."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    s = np.asarray(sign)
    ru = raw_ids(n_u, 0)[u] if remap else u
    rv = raw_ids(n_v, 1)[v] if remap else v
    wu = max(1, len(str(int(ru.max())))) if ru.size else 1
    wv = max(1, len(str(int(rv.max())))) if rv.size else 1
    m = u.shape[0]
    line = np.empty((m, wu + wv + 4), np.uint8)
    line[:, :wu] = _digits(ru, wu)
    line[:, wu] = ord(" ")
    line[:, wu + 1:wu + 1 + wv] = _digits(rv, wv)
    line[:, wu + 1 + wv] = ord(" ")
    line[:, wu + 2 + wv] = np.where(s < 0, ord("0"), ord("1")).astype(np.uint8)
    line[:, wu + 3 + wv] = ord("\n")
    return line.tobytes()


def messy_edge_text(n_u: int, n_v: int, u, v, sign, seed: int = 0) -> tuple[bytes, list[int]]:
    """The same records with random formatting choices per line, comment and
    blank lines in between, and the returned list of the line numbers (from
    1) that hold the records, in record order."""
    rng = np.random.default_rng(seed)
    ru = raw_ids(n_u, 0)[np.asarray(u, np.int64)]
    rv = raw_ids(n_v, 1)[np.asarray(v, np.int64)]
    seps = [" ", "\t", ",", "  ", " \t", ", "]
    lines, rec_lines = [], []
    for a, b, s in zip(ru.tolist(), rv.tolist(), np.asarray(sign).tolist()):
        r = rng.random()
        if r < 0.05:
            lines.append("% a comment line")
        elif r < 0.08:
            lines.append("   # another comment 1 2 1")
        elif r < 0.11:
            lines.append(rng.choice(["", "   ", "\t"]))
        sep1, sep2 = rng.choice(seps), rng.choice(seps)
        if s < 0:
            tok = rng.choice(["0", "-1"])
        else:
            tok = rng.choice(["1", "+1"])
        a_s = ("0" * int(rng.integers(0, 3))) + str(a)
        lead = rng.choice(["", " ", "\t"])
        tail = rng.choice(["", " ", " 12345 extra", "\t3.5"])
        lines.append(f"{lead}{a_s}{sep1}{b}{sep2}{tok}{tail}")
        rec_lines.append(len(lines))
    ends = ["\r\n" if rng.random() < 0.3 else "\n" for _ in lines]
    text = "".join(line + e for line, e in zip(lines, ends))
    if rng.random() < 0.5 and text.endswith("\n"):
        text = text.rstrip("\r\n")
    return text.encode(), rec_lines

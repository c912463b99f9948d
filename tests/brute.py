"""Pure-Python brute force of the oracle's definitions, for tiny inputs only.

An independent restatement in Python integers (floor division ``//``) and
``math.fsum``; it checks the oracle's loops, indexing, pass order and
aggregation.  The transform matrix is taken from the oracle, whose entries are
pinned separately against the orthonormal DCT-II and its structure.
"""
import math


def shifts(w, bit_depth):
    lw = w.bit_length() - 1
    return lw + bit_depth - 9, lw + 6


def block_coeffs(X, C, w, K, bit_depth):
    """X: w x w list of ints (raw samples); returns the K x K coefficient list."""
    s1, s2 = shifts(w, bit_depth)
    T = [[(sum(X[m][n] * C[k][n] for n in range(w)) + (1 << (s1 - 1))) // (1 << s1)
          for k in range(K)] for m in range(w)]
    return [[(sum(C[i][m] * T[m][k] for m in range(w)) + (1 << (s2 - 1))) // (1 << s2)
             for k in range(K)] for i in range(K)]


def weight(i, j, w):
    return math.exp(abs(((i + 1) * (j + 1) / (w * w)) ** 2 - 1.0))


def block_energy(Y, w):
    K = len(Y)
    return math.fsum(weight(i, k, w) * abs(Y[i][k]) for i in range(K) for k in range(K)
                     if (i, k) != (0, 0))


def plane_blocks(plane, w):
    """Complete w x w blocks of a 2-D list, raster order."""
    H, W = len(plane), len(plane[0])
    for by in range(H // w):
        for bx in range(W // w):
            yield [[int(plane[by * w + m][bx * w + n]) for n in range(w)] for m in range(w)]


def features(frames, C, w, K, bit_depth):
    """frames: list of (Y, U, V) 2-D lists.  Returns (features, block H lists)."""
    out, Hs = [], []
    prev = None
    for (Yp, Up, Vp) in frames:
        Hf, Lf = [], []
        for plane in (Yp, Up, Vp):
            hs, ls = [], []
            for X in plane_blocks(plane, w):
                Yc = block_coeffs(X, C, w, K, bit_depth)
                hs.append(block_energy(Yc, w))
                ls.append(math.sqrt(Yc[0][0]))
            Hf.append(hs)
            Lf.append(ls)
        ww = w * w
        E = [math.fsum(h) / (len(h) * ww) for h in Hf]
        L = [math.fsum(l) / (len(l) * ww) for l in Lf]
        if prev is None:
            hfeat = 0.0
        else:
            hfeat = math.fsum(abs(a - b) for a, b in zip(Hf[0], prev)) / (len(Hf[0]) * ww)
        prev = Hf[0]
        out.append([E[0], hfeat, L[0], E[1], E[2], L[1], L[2]])
        Hs.append(Hf[0] + Hf[1] + Hf[2])
    return out, Hs

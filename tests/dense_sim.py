"""Dense state-vector simulator of the walk on tiny registers (test pin).

Independent of the oracle: the full register space (j_c, j, b1, k_c, k, b2)
of 2^(4n+2) amplitudes is held as one dense numpy vector whose flat index is
the packed key [j_c | j | b1 | k_c | k | b2].  Each operator is built as a
permutation, a block of small dense matrices or a sign, without an explicit
data register: the three QRAM reads of Alg. 5 (O_A' compute, rotation,
O_A' uncompute around O_s' / O_s'^dagger) collapse into one rotation on b2
applied in the (l, z) frame, controlled by the row j, the slot l and the
column register value z ^ k_{j,l}.

Preprocessing is written out again here (scale by 1/max(1, max|a|), s = next
power of two of the largest column count, filler rows = smallest missing
indices with value 0) so that nothing is taken from the oracle.
"""
from __future__ import annotations

import math

import numpy as np


def preprocess(csc, scale=None):
    n = csc.n
    nbits = max(1, int(np.ceil(np.log2(n))))
    N = 1 << nbits
    counts = np.diff(csc.colptr)
    s = 1 << int(np.ceil(np.log2(max(1, counts.max()))))
    if scale is None:
        scale = 1.0 / max(1.0, np.abs(csc.vals).max())
    col = np.zeros((N, s), np.int64)
    val = np.zeros((N, s), dtype=csc.vals.dtype)
    for c in range(N):
        rows = list(csc.rowidx[csc.colptr[c]:csc.colptr[c + 1]]) if c < n else []
        vals = list(csc.vals[csc.colptr[c]:csc.colptr[c + 1]] * scale) if c < n else []
        present = set(rows)
        r = 0
        while len(rows) < s:
            if r not in present:
                rows.append(r)
                vals.append(0.0)
            r += 1
        order = np.argsort(rows)
        col[c] = np.asarray(rows)[order]
        val[c] = np.asarray(vals)[order]
    return N, nbits, s, scale, col, val


def _position(col, j, k):
    row = col[j]
    hit = np.nonzero(row == k)[0]
    return int(hit[0]) if hit.size else 0


def fixed_point_rotation(a, w, row, column):
    """(f, g) for the real value a = +-q / 2^w of fixed-point data, written
    out from the definitions: the square-root register is sqrt(q / 2^w)
    truncated to w fraction bits, the angle register the arccos of that in
    units of (pi/2) / 2^w rounded to the nearest integer, and the rotation is
    by that angle (f = cos, times +-i by the order of row and column for a
    negative value; g = sin)."""
    q = int(round(abs(a) * 2 ** w))
    assert q == abs(a) * 2 ** w and q < 2 ** w, "not a fixed-point value"
    r = math.isqrt(q << w)
    t = round(math.acos(r / 2 ** w) * 2 ** (w + 1) / math.pi)
    if t == 2 ** w:
        c, sn = 0.0, 1.0
    elif t == 0:
        c, sn = 1.0, 0.0
    else:
        theta = math.pi / 2 * t / 2 ** w
        c, sn = math.cos(theta), math.sin(theta)
    if math.copysign(1.0, a) > 0 or q == 0:
        return complex(c, 0.0), sn
    return (1j if row <= column else -1j) * c, sn


class DenseWalk:
    """``jc_dim``: number of values of register j_c held (default N).  Every
    state reachable from |b~> or T~|b~> has j_c < s at all times and k_c < s
    at step boundaries (k_c holds z < N only inside T~^dagger ... T~), so
    jc_dim = s keeps the whole walk while cutting the vector by N/s; j_c is
    the most significant register, so the flat index still equals the packed
    key.  S then moves only entries with k_c < jc_dim and asserts that the
    others are zero."""

    def __init__(self, csc, scale=None, word=0, jc_dim=None):
        self.N, self.n, self.s, self.scale, self.col, self.val = preprocess(csc, scale)
        N, s = self.N, self.s
        self.jc_dim = N if jc_dim is None else int(jc_dim)
        self.shape = (self.jc_dim, N, 2, N, N, 2)
        self.size = int(np.prod(self.shape))
        c = np.indices(self.shape).reshape(6, -1)
        jc, j, b1, kc, k, b2 = c
        flat = lambda *a: np.ravel_multi_index(a, self.shape)
        # position table pos[j, k] = i_j(k)
        pos = np.zeros((N, N), np.int64)
        for r in range(N):
            for x in range(N):
                pos[r, x] = _position(self.col, r, x)
        # O_s': (l in k, z in k_c) -> (k, k_c) for l < s; registers swapped for l >= s
        valid = k < s
        knew = np.where(valid, kc ^ self.col[j, np.minimum(k, s - 1)], kc)
        kcnew = np.where(valid, k ^ pos[j, knew], k)
        self.os_perm = flat(jc, j, b1, kcnew, knew, b2)
        assert np.unique(self.os_perm).size == self.size
        s_ok = kc < self.jc_dim
        self.s_full = bool(s_ok.all())
        if self.s_full:
            self.s_perm = flat(kc, k, b2, jc, j, b1)
        else:
            self.s_src = np.nonzero(s_ok)[0]
            self.s_dst = flat(kc[s_ok], k[s_ok], b2[s_ok], jc[s_ok], j[s_ok], b1[s_ok])
            self.s_drop = np.nonzero(~s_ok)[0]
        self.p_sign = np.where((jc == 0) & (b1 == 0) & (kc == 0) & (k == 0) & (b2 == 0), 1.0, -1.0)
        # rotation in the (l, z) frame: controlled by j, l = k register, z = k_c register
        ll = np.minimum(k, s - 1)
        a = self.val[j, ll]
        colk = kc ^ self.col[j, ll]
        # real values: sqrt(a) for a >= 0, +-i sqrt|a| by the order of row and
        # column for a < 0; values off the real axis: the principal sqrt(a)
        ar, ai = np.real(a), np.imag(a)
        f_real = np.where(ar >= 0, np.sqrt(np.abs(ar)) + 0j, np.where(j <= colk, 1j, -1j) * np.sqrt(np.abs(ar)))
        f = np.where(ai != 0, np.sqrt(a + 0j), f_real)
        g = np.sqrt(1.0 - np.abs(a))
        if word:
            # fixed-point data: one rotation per (value, row, column) triple
            table = {}
            f = np.empty(a.shape, complex)
            g = np.empty(a.shape)
            for idx, (av, jv, cv) in enumerate(zip(ar.tolist(), j.tolist(), colk.tolist())):
                key = (av, jv <= cv)
                if key not in table:
                    table[key] = fixed_point_rotation(av, word, jv, cv)
                f[idx], g[idx] = table[key]
        self.rot_valid = valid
        self.f, self.g = f, g
        # per amplitude pair (f, g and the slot range do not depend on b2)
        self.f2, self.g2, self.valid2 = f[0::2], g[0::2], valid[0::2]
        self.b2 = b2
        self.partner = flat(jc, j, b1, kc, k, 1 - b2)
        hs = np.array([[1.0]])
        while hs.shape[0] < s:
            hs = np.block([[hs, hs], [hs, -hs]])
        self.hmat = hs / np.sqrt(s)

    # --- operators on a dense vector
    def OS(self, psi):
        out = np.zeros_like(psi)
        out[self.os_perm] = psi
        return out

    def OSinv(self, psi):
        return psi[self.os_perm]

    def S(self, psi):
        out = np.zeros_like(psi)
        if self.s_full:
            out[self.s_perm] = psi
        else:
            if np.any(psi[self.s_drop] != 0):
                raise AssertionError("k_c >= jc_dim at S: the restricted register range does not hold the walk")
            out[self.s_dst] = psi[self.s_src]
        return out

    def P(self, psi):
        return psi * self.p_sign

    def H(self, psi):
        # H on each of the low log2(s) bits of k in turn: (v0, v1) -> (v0 + v1,
        # v0 - v1) on the pairs that differ in that bit, then 1/sqrt(s) once
        s = self.s
        out = psi * (1.0 / np.sqrt(s))
        h = 1
        while h < s:
            # (registers above, higher bits of k, this bit, lower bits of k, b2)
            v = out.reshape(-1, s // (2 * h), 2, h, 2)
            d = v[:, :, 0] - v[:, :, 1]
            v[:, :, 0] += v[:, :, 1]
            v[:, :, 1] = d
            h *= 2
        return out

    def R(self, psi, dagger=False):
        # b2 is the lowest register: amplitude pairs (b2 = 0, b2 = 1)
        x = psi.reshape(-1, 2)
        v0, v1 = x[:, 0], x[:, 1]
        f, g = self.f2, self.g2
        if not dagger:
            # [[f, -g], [g, conj f]]
            o0, o1 = f * v0 - g * v1, g * v0 + np.conj(f) * v1
        else:
            # [[conj f, g], [-g, f]]
            o0, o1 = np.conj(f) * v0 + g * v1, -g * v0 + f * v1
        if np.any(~self.valid2[:, None] & (x != 0)):
            raise AssertionError("amplitude outside the slot range at a rotation")
        return np.where(self.valid2[:, None], np.stack((o0, o1), axis=1), x).reshape(-1)

    def T(self, psi):
        return self.OS(self.R(self.H(psi)))

    def Tdag(self, psi):
        return self.H(self.R(self.OSinv(psi), dagger=True))

    def W(self, psi):
        return self.S(self.T(self.P(self.Tdag(psi))))

    def basis_b(self, b):
        psi = np.zeros(self.size, complex)
        for j, bj in enumerate(b):
            psi[np.ravel_multi_index((0, j, 0, 0, 0, 0), self.shape)] = bj
        return psi


def torch_loss(csc, vals_scaled, b, w, nsteps, scale=1.0):
    """Same dense walk written with torch ops, differentiable in the stored
    (already scaled) CSC values (real, or complex for a complex matrix) and in b.  Returns (loss, vals tensor, b tensor).
    Loss = sum_j w_j p_j with p the marginal of register j after
    W^nsteps T~ |b~>."""
    import torch

    dw = DenseWalk(csc, scale=scale)
    N, s = dw.N, dw.s
    cplx = np.iscomplexobj(vals_scaled)
    vdt = torch.complex128 if cplx else torch.float64
    v = torch.tensor(np.asarray(vals_scaled, dtype=np.complex128 if cplx else np.float64), requires_grad=True)
    bt = torch.tensor(np.asarray(b, dtype=np.complex128), requires_grad=True)
    # ELL value table as a differentiable gather of the CSC values
    slot_of = np.full((N, s), -1, np.int64)
    for c in range(csc.n):
        for p in range(csc.colptr[c], csc.colptr[c + 1]):
            l = int(np.nonzero(dw.col[c] == csc.rowidx[p])[0][0])
            slot_of[c, l] = p
    ell = torch.zeros(N * s, dtype=vdt)
    idx = np.nonzero(slot_of.reshape(-1) >= 0)[0]
    ell = ell.index_put((torch.tensor(idx),), v[torch.tensor(slot_of.reshape(-1)[idx])])
    ell = ell.reshape(N, s)
    c = np.indices(dw.shape).reshape(6, -1)
    jc, j, b1, kc, k, b2 = c
    ll = np.minimum(k, s - 1)
    a = ell[torch.tensor(j), torch.tensor(ll)]
    colk = kc ^ dw.col[j, ll]
    neg_phase = np.where(j <= colk, 1j, -1j)
    if cplx:
        # the principal sqrt(a) off the negative real axis, the +-i rule on it
        cut = (a.imag == 0) & (a.real < 0)
        f_rule = torch.sqrt(torch.abs(a)) * torch.tensor(neg_phase, dtype=torch.complex128)
        f = torch.where(cut, f_rule, torch.sqrt(torch.where(cut, torch.ones_like(a), a)))
    else:
        phase = torch.where(a >= 0, torch.ones_like(a, dtype=torch.complex128),
                            torch.tensor(neg_phase, dtype=torch.complex128))
        f = torch.sqrt(torch.abs(a)) * phase
    g = torch.sqrt(1.0 - torch.abs(a)).to(torch.complex128)
    valid = torch.tensor(dw.rot_valid)
    b2t = torch.tensor(dw.b2)
    partner = torch.tensor(dw.partner)
    os_perm = torch.tensor(dw.os_perm)
    s_perm = torch.tensor(dw.s_perm)
    p_sign = torch.tensor(dw.p_sign, dtype=torch.complex128)
    hmat = torch.tensor(dw.hmat, dtype=torch.complex128)

    def R(psi, dagger):
        wv = psi[partner]
        if not dagger:
            new = torch.where(b2t == 0, f * psi - g * wv, g * wv + torch.conj(f) * psi)
        else:
            new = torch.where(b2t == 0, torch.conj(f) * psi + g * wv, -g * wv + f * psi)
        return torch.where(valid, new, psi)

    def H(psi):
        x = psi.reshape(N, N, 2, N, N // s, s, 2)
        return torch.einsum("xy,abcdeyg->abcdexg", hmat, x).reshape(-1)

    def OS(psi):
        return torch.zeros_like(psi).index_put((os_perm,), psi)

    def OSinv(psi):
        return psi[os_perm]

    def S(psi):
        return torch.zeros_like(psi).index_put((s_perm,), psi)

    psi = torch.zeros(dw.size, dtype=torch.complex128)
    jidx = torch.tensor([np.ravel_multi_index((0, jj, 0, 0, 0, 0), dw.shape) for jj in range(len(b))])
    psi = psi.index_put((jidx,), bt)
    psi = OS(R(H(psi), False))
    for _ in range(nsteps):
        t = H(R(OSinv(psi), True))
        t = t * p_sign
        t = OS(R(H(t), False))
        psi = S(t)
    prob = (psi.real ** 2 + psi.imag ** 2).reshape(N, N, 2, N, N, 2).sum(dim=(0, 2, 3, 4, 5))
    wt = torch.zeros(N, dtype=torch.float64)
    wt[:len(w)] = torch.tensor(np.asarray(w, dtype=np.float64))
    loss = (prob * wt).sum()
    return loss, v, bt

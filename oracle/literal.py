"""A second, independent transcription of the synchronous 2D decoder.

TEST INFRASTRUCTURE ONLY.  Pure Python with sets, dictionaries and loops, for
tiny lattices (L <= 8), written from the definitions without reference to the
C oracle in this folder, so that the two can be checked against each other
pattern by pattern.  It shares no code with the C oracle or the HIP library.

Notation follows the paper:
  * sites r = (x, y) of the L x L torus, syndrome sigma_r in {+1, -1};
  * registers m^{sa}_r for s in {+1, -1} and axis a in {1, 2} (1 = x, 2 = y);
  * one decoder step is Phi_F o Phi_A^v (Def. "synchronous automaton
    decoder"), with A^{(D)} and F^{(D)} of Def. "message passing automaton,
    general dimensions" (Sec. 3.2) and the OR function of Def. "message
    passing automaton, 1D".

Readings (the same choices the decoder makes everywhere, stated with it):
  * C^{(a)}_r is the set of the three sites r + k b-hat, k in {-1, 0, 1},
    b the axis normal to a;
  * the "min + 1" branch of A^{(D)} minimises over the nonzero registers;
  * argmin' compares the message values first and uses s a/(D+1) only to
    order equal values;
  * f^a = sgn(m^{-a} - m^{+a}) reads an absent message as +infinity (the
    anyon moves toward the source of its smallest message; no move on an
    exact tie on that axis);
  * only anyon sites (sigma = -1) carry a force.
"""
from __future__ import annotations

V = 3
DIRECTIONS = [(+1, 1), (-1, 1), (+1, 2), (-1, 2)]  # (s, a): +x, -x, +y, -y


def unit(a):
    return (1, 0) if a == 1 else (0, 1)


def add(L, r, d, k=1):
    return ((r[0] + k * d[0]) % L, (r[1] + k * d[1]) % L)


def C(L, r, a):
    """C^{(a)}_r: the unit infinity-ball around r in the directions normal to a-hat."""
    b = unit(2 if a == 1 else 1)
    return {add(L, r, b, k) for k in (-1, 0, 1)}


def A_ct(sigma, S):
    """1 if some site of S holds an anyon."""
    return 1 if any(sigma[q] == -1 for q in S) else 0


def sgn(z):
    return (z > 0) - (z < 0)


class Decoder:
    def __init__(self, L, ex, ey):
        """ex[(x, y)] = error on link (x,y)-(x+1,y); ey[(x, y)] on (x,y)-(x,y+1)."""
        self.L = L
        self.sites = [(x, y) for y in range(L) for x in range(L)]
        self.E = {("x", r): ex.get(r, 0) for r in self.sites}
        self.E.update({("y", r): ey.get(r, 0) for r in self.sites})
        self.Cor = {k: 0 for k in self.E}
        self.sigma = {}
        for r in self.sites:
            touched = (self.E[("x", r)] + self.E[("x", add(L, r, (-1, 0)))]
                       + self.E[("y", r)] + self.E[("y", add(L, r, (0, -1)))])
            self.sigma[r] = -1 if touched % 2 else +1
        self.m = {d: {r: 0 for r in self.sites} for d in DIRECTIONS}
        self.t = 0

    def anyons(self):
        return {r for r in self.sites if self.sigma[r] == -1}

    # ---- A^{(D)}: one synchronous message update
    def message_update(self):
        L = self.L
        new = {}
        for (s, a) in DIRECTIONS:
            col = {}
            for r in self.sites:
                S = C(L, add(L, r, unit(a), -s), a)  # C^{(a)}_{r - s a}
                if A_ct(self.sigma, S):
                    col[r] = 1
                else:
                    nz = [self.m[(s, a)][q] for q in S if self.m[(s, a)][q] > 0]
                    col[r] = min(nz) + 1 if nz else 0
            new[(s, a)] = col
        self.m = new

    # ---- F^{(D)}: forces, OR'd link exponents, flips
    def forces(self):
        f = {}
        for r in self.sites:
            f[r] = {1: 0, 2: 0}
            if self.sigma[r] != -1:
                continue
            M = [(s, a) for (s, a) in DIRECTIONS if self.m[(s, a)][r] > 0]
            if not M:
                continue
            s_r, a_r = min(M, key=lambda sa: (self.m[sa][r], sa[0] * sa[1]))
            inf = float("inf")
            mp = self.m[(+1, a_r)][r] or inf
            mm = self.m[(-1, a_r)][r] or inf
            f[r][a_r] = sgn(mm - mp) if mp != mm else 0
        return f

    def feedback(self):
        L = self.L
        f = self.forces()
        flips = []
        for r in self.sites:
            for a, name in ((1, "x"), (2, "y")):
                r2 = add(L, r, unit(a))
                x = self.sigma[r] * f[r][a]
                y = self.sigma[r2] * (-f[r2][a])
                if x == 1 or y == 1:  # the OR function
                    flips.append((name, r))
        for name, r in flips:
            self.Cor[(name, r)] ^= 1
            r2 = add(L, r, unit(1 if name == "x" else 2))
            self.sigma[r] = -self.sigma[r]
            self.sigma[r2] = -self.sigma[r2]

    def step(self):
        for _ in range(V):
            self.message_update()
        self.t += 1
        self.feedback()

    def windings(self):
        """Parities of E + C across the cuts x = L-1 (x-links) and y = L-1 (y-links)."""
        L = self.L
        wx = sum(self.E[("x", (L - 1, y))] ^ self.Cor[("x", (L - 1, y))] for y in range(L)) % 2
        wy = sum(self.E[("y", (x, L - 1))] ^ self.Cor[("y", (x, L - 1))] for x in range(L)) % 2
        return wx, wy


def decode(L, ex, ey, T_max):
    """Returns (T_dec, flags, anyon set, registers) with flags bit 0 = logical
    failure, bit 1 = timeout (anyons left after T_max steps, counted as a
    failure)."""
    d = Decoder(L, ex, ey)
    while d.anyons() and d.t < T_max:
        d.step()
    timeout = bool(d.anyons())
    wx, wy = d.windings()
    fail = timeout or wx == 1 or wy == 1
    return d.t, (1 if fail else 0) | (2 if timeout else 0), d.anyons(), d.m


def run(L, ex, ey, t_exact):
    """Exactly t_exact steps; returns the decoder."""
    d = Decoder(L, ex, ey)
    for _ in range(t_exact):
        d.step()
    return d

"""Naive NumPy transcription of the FRE LBM step for tiny lattices.

TEST INFRASTRUCTURE ONLY.  A second, independently structured rendering of
the same step as ``frelbm_oracle.c`` (Sec. 2.2-2.3 and Algorithm 1 of Simonis
et al., arXiv 2212.01617, with the readings listed at the top of that file):
whole-array NumPy expressions over a padded grid, equilibria written in the
expanded form w rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u], explicit neighbour
tables, and pull-form bookkeeping of the bounce-back.  It exists to catch
transcription slips (a wrong index, sign or weight) in the C oracle.
"""
from __future__ import annotations

import numpy as np

D2Q9 = (
    np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0]]),
    np.array([16, 4, 4, 4, 4, 1, 1, 1, 1]) / 36.0,
)
D3Q19 = (
    np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
              [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]]),
    np.array([12] + [2] * 6 + [1] * 12) / 36.0,
)


class Brute:
    """State on the padded grid (ghost layer on wall axes)."""

    def __init__(self, kind, shape_xyz, phi0, rho0=None, u0=None, mask=None, *,
                 bc=(0, 0, 0), wall_u=None, rollers=(), kappa1, kappa2, alpha,
                 tau_f, tau_g, M):
        self.c, self.w = D2Q9 if kind == 0 else D3Q19
        self.q = len(self.w)
        self.opp = np.array([int(np.where((self.c == -self.c[i]).all(1))[0][0])
                             for i in range(self.q)])
        nx, ny, nz = shape_xyz
        self.n = np.array([nx, ny, nz])
        self.bc = np.array(bc)
        self.pad = (self.bc == 1).astype(int)
        self.ext = self.n + 2 * self.pad
        self.wall_u = np.zeros((3, 2, 3)) if wall_u is None else np.asarray(wall_u, float)
        self.rollers = list(rollers)
        self.k1, self.k2, self.al = kappa1, kappa2, alpha
        self.tf, self.tg = tau_f, tau_g
        self.Gamma = M / (tau_g - 0.5)
        E = int(np.prod(self.ext))
        self.E = E
        # coordinates of every extended cell, index = x + ex*(y + ey*z)
        ex, ey, ez = self.ext
        zz, yy, xx = np.meshgrid(np.arange(ez), np.arange(ey), np.arange(ex), indexing="ij")
        self.xyz = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
        # cell kinds
        code = np.full(E, 8, dtype=np.int64)
        inner = np.all((self.xyz >= self.pad) & (self.xyz < self.pad + self.n), axis=1)
        user = self.xyz[inner] - self.pad
        uidx = user[:, 0] + nx * (user[:, 1] + ny * user[:, 2])
        m = np.zeros(nx * ny * nz, dtype=np.int64) if mask is None else np.asarray(mask).reshape(-1)
        code[inner] = m[uidx]
        self.code = code
        self.fluid = code == 0
        self.inner_idx = np.nonzero(inner)[0]
        self.user_of_inner = uidx
        # neighbour table nb[i, cell] (-1 beyond a wall axis)
        nb = np.empty((self.q, E), dtype=np.int64)
        for i in range(self.q):
            p = self.xyz + self.c[i]
            ok = np.ones(E, bool)
            for a in range(3):
                if self.bc[a] == 0:
                    p[:, a] %= self.ext[a]
                else:
                    ok &= (p[:, a] >= 0) & (p[:, a] < self.ext[a])
            lin = p[:, 0] + ex * (p[:, 1] + ey * p[:, 2])
            nb[i] = np.where(ok, lin, -1)
        self.nb = nb
        # initial fields
        N = nx * ny * nz
        def to_ext(v, default):
            out = np.zeros(E)
            vv = np.full(N, default) if v is None else np.asarray(v, float).reshape(-1)
            out[self.inner_idx] = vv[self.user_of_inner]
            return out * self.fluid
        phi = to_ext(phi0, 0.0)
        rho = to_ext(rho0, 1.0)
        u = np.zeros((3, E))
        if u0 is not None:
            uu = np.asarray(u0, float).reshape(3, -1)
            for a in range(3):
                u[a] = to_ext(uu[a], 0.0)
        mur, mup = self._potentials(rho, phi)
        self.f = self._feq(rho, u)
        self.g = self._geq(phi, mup, u)
        self.t = 0

    # -- helpers -----------------------------------------------------------
    def _fill(self, X):
        """solid cells <- weighted mean of fluid neighbours"""
        X = X * self.fluid
        num = np.zeros(self.E)
        den = np.zeros(self.E)
        for i in range(1, self.q):
            nbi = self.nb[i]
            ok = nbi >= 0
            fl = np.zeros(self.E, bool)
            fl[ok] = self.fluid[nbi[ok]]
            num[fl] += self.w[i] * X[nbi[fl]]
            den[fl] += self.w[i]
        solid = ~self.fluid
        out = X.copy()
        with np.errstate(invalid="ignore", divide="ignore"):
            out[solid] = np.where(den[solid] > 0, num[solid] / den[solid], 0.0)
        return out

    def _lap(self, X):
        acc = np.zeros(self.E)
        F = np.nonzero(self.fluid)[0]
        for i in range(1, self.q):
            acc[F] += self.w[i] * (X[self.nb[i, F]] - X[F])
        return 6.0 * acc

    def _grad(self, X):
        g = np.zeros((3, self.E))
        F = np.nonzero(self.fluid)[0]
        for i in range(self.q):
            for a in range(3):
                if self.c[i, a]:
                    g[a, F] += 3.0 * self.w[i] * self.c[i, a] * X[self.nb[i, F]]
        return g

    def _potentials(self, rho, phi):
        rt, pt = self._fill(rho), self._fill(phi)
        lr, lp = self._lap(rt), self._lap(pt)
        s, t = rho + phi, rho - phi
        cub_s = s * (s - 1) * (s - 2)
        cub_t = t * (t - 1) * (t - 2)
        a2 = self.al ** 2
        mur = self.k1 / 8 * cub_s + self.k2 / 8 * cub_t \
            - a2 / 4 * (self.k1 + self.k2) * lr + a2 / 4 * (self.k2 - self.k1) * lp
        mup = self.k1 / 8 * cub_s - self.k2 / 8 * cub_t \
            - a2 / 4 * (self.k1 + self.k2) * lp + a2 / 4 * (self.k2 - self.k1) * lr
        return mur * self.fluid, mup * self.fluid

    def _feq(self, rho, u):
        cu = self.c @ u  # (q, E)
        uu = (u * u).sum(0)
        return self.w[:, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu) * self.fluid

    def _geq(self, phi, mup, u):
        cu = self.c @ u
        uu = (u * u).sum(0)
        g = self.w[:, None] * (3 * self.Gamma * mup + phi * (3 * cu + 4.5 * cu ** 2 - 1.5 * uu))
        g[0] = phi - g[1:].sum(0)
        return g * self.fluid

    def _body_u(self, x_cell, s_cell, i):
        """velocity of the body owning solid s at the link midpoint"""
        code = self.code[s_cell]
        if code == 1:
            return np.zeros(3)
        if code == 8:
            p = self.xyz[s_cell]
            acc, n = np.zeros(3), 0
            for a in range(3):
                if self.bc[a] != 1:
                    continue
                if p[a] == 0:
                    acc += self.wall_u[a, 0]; n += 1
                elif p[a] == self.ext[a] - 1:
                    acc += self.wall_u[a, 1]; n += 1
            return acc / max(n, 1)
        cen, om, ax = self.rollers[code - 2]
        mid = self.xyz[x_cell] - self.pad + 0.5 * self.c[i]
        d = mid - np.asarray(cen, float)
        axis = np.zeros(3); axis[ax] = 1.0
        return om * np.cross(axis, d)

    # -- step --------------------------------------------------------------
    def step(self, n=1):
        for _ in range(n):
            self._step()
        return self

    def _moments(self):
        rho = self.f.sum(0) * self.fluid
        phi = self.g.sum(0) * self.fluid
        j = (self.c.T @ self.f) * self.fluid
        mur, mup = self._potentials(rho, phi)
        # eq. (F) through the product rule:
        #   -rho grad mu_rho - phi grad mu_phi
        #     = mu_rho grad rho + mu_phi grad phi - grad(rho mu_rho + phi mu_phi)
        pi = rho * mur + phi * mup
        F = (mur * self._grad(self._fill(rho)) + mup * self._grad(self._fill(phi))
             - self._grad(self._fill(pi))) * self.fluid
        with np.errstate(invalid="ignore", divide="ignore"):
            u = np.where(self.fluid, (j + 0.5 * F) / np.where(self.fluid, rho, 1.0), 0.0)
        return rho, phi, j, mur, mup, F, u

    def _step(self):
        rho, phi, j, mur, mup, F, u = self._moments()
        cu = self.c @ u
        cF = self.c @ F
        uF = (u * F).sum(0)
        S = (1 - 0.5 / self.tf) * self.w[:, None] * (3 * (cF - uF) + 9 * cu * cF)
        fs = self.f - (self.f - self._feq(rho, u)) / self.tf + S
        gs = self.g - (self.g - self._geq(phi, mup, u)) / self.tg
        fn = np.zeros_like(self.f)
        gn = np.zeros_like(self.g)
        F_idx = np.nonzero(self.fluid)[0]
        for i in range(self.q):
            # pull: f_i(x, t+1) = f_i*(x - c_i) if that is fluid, else the
            # bounced population of direction opp(i) at x
            io = self.opp[i]
            src = self.nb[io, F_idx]  # x - c_i
            fl = self.fluid[src]
            fn[i, F_idx[fl]] = fs[i, src[fl]]
            gn[i, F_idx[fl]] = gs[i, src[fl]]
            for x, s in zip(F_idx[~fl], src[~fl]):
                uw = self._body_u(x, s, io)
                cw = self.c[io] @ uw
                fn[i, x] = fs[io, x] - 6 * self.w[io] * rho[x] * cw
                gn[i, x] = gs[io, x] - 6 * self.w[io] * phi[x] * cw
        self.f, self.g = fn, gn
        self.t += 1

    # -- output ------------------------------------------------------------
    def _user(self, X):
        out = np.zeros(int(np.prod(self.n)))
        out[self.user_of_inner] = X[self.inner_idx]
        nx, ny, nz = self.n
        return out.reshape(nz, ny, nx)

    def observe(self):
        rho, phi, j, mur, mup, F, u = self._moments()
        return {"rho": self._user(rho), "phi": self._user(phi),
                "ux": self._user(u[0]), "uy": self._user(u[1]), "uz": self._user(u[2]),
                "mu_rho": self._user(mur), "mu_phi": self._user(mup)}

    def populations(self):
        return (np.stack([self._user(self.f[i]) for i in range(self.q)]),
                np.stack([self._user(self.g[i]) for i in range(self.q)]))


class Brute3(Brute):
    """The ternary step (Sec. 2.2, Remark after the mobility relation) in the
    same naive form, written in the concentrations C1 = (rho + phi - psi)/2,
    C2 = (rho - phi - psi)/2, C3 = psi of the cited ternary free energy
    sum_m kappa_m/2 C_m^2 (1 - C_m)^2 + alpha^2 kappa_m/2 |grad C_m|^2: the
    potential of each concentration, mu_m = kappa_m C_m (1 - C_m)(1 - 2 C_m)
    - alpha^2 kappa_m lap C_m, and the force sum_m mu_m grad C_m - grad(sum_m
    C_m mu_m), equal to the form in (rho, phi, psi) of the C oracle by the
    chain rule; the third population h relaxes like g towards the equilibrium
    with (psi, mu_psi, Gamma_psi)."""

    def __init__(self, kind, shape_xyz, phi0, psi0, rho0=None, u0=None, mask=None, *, kappa3, M3, tau_h, **kw):
        self.k3, self.th = kappa3, tau_h
        self.G3 = M3 / (tau_h - 0.5)
        self._psi0 = psi0
        super().__init__(kind, shape_xyz, phi0, rho0, u0, mask, **kw)
        # the base class set f and g from the binary potentials: redo all
        # three from the ternary ones
        nx, ny, nz = self.n
        N = nx * ny * nz
        def to_ext(v, default):
            out = np.zeros(self.E)
            vv = np.full(N, default) if v is None else np.asarray(v, float).reshape(-1)
            out[self.inner_idx] = vv[self.user_of_inner]
            return out * self.fluid
        phi, psi, rho = to_ext(phi0, 0.0), to_ext(psi0, 0.0), to_ext(rho0, 1.0)
        u = np.zeros((3, self.E))
        if u0 is not None:
            uu = np.asarray(u0, float).reshape(3, -1)
            for a in range(3):
                u[a] = to_ext(uu[a], 0.0)
        mur, mup, muq = self._potentials3(rho, phi, psi)
        self.f = self._feq(rho, u)
        self.g = self._geq(phi, mup, u)
        self.h = self._heq(psi, muq, u)

    def _heq(self, psi, muq, u):
        cu = self.c @ u
        uu = (u * u).sum(0)
        h = self.w[:, None] * (3 * self.G3 * muq + psi * (3 * cu + 4.5 * cu ** 2 - 1.5 * uu))
        h[0] = psi - h[1:].sum(0)
        return h * self.fluid

    def _conc(self, rho, phi, psi):
        return [0.5 * (rho + phi - psi), 0.5 * (rho - phi - psi), psi]

    def _mu_conc(self, rho, phi, psi):
        """potential of each concentration at fluid cells"""
        Cs = self._conc(self._fill(rho), self._fill(phi), self._fill(psi))
        Cr = self._conc(rho, phi, psi)
        out = []
        for k, C, Cf in zip((self.k1, self.k2, self.k3), Cr, Cs):
            out.append((k * C * (1 - C) * (1 - 2 * C) - self.al ** 2 * k * self._lap(Cf)) * self.fluid)
        return out

    def _potentials3(self, rho, phi, psi):
        m1, m2, m3 = self._mu_conc(rho, phi, psi)
        return 0.5 * (m1 + m2), 0.5 * (m1 - m2), m3 - 0.5 * (m1 + m2)

    def _moments3(self):
        rho = self.f.sum(0) * self.fluid
        phi = self.g.sum(0) * self.fluid
        psi = self.h.sum(0) * self.fluid
        j = (self.c.T @ self.f) * self.fluid
        mu = self._mu_conc(rho, phi, psi)
        Cr = self._conc(rho, phi, psi)
        pi = sum(C * m for C, m in zip(Cr, mu))
        F = -self._grad(self._fill(pi))
        for C, m in zip(Cr, mu):
            # grad of the filled concentration: the fill is linear, so this is
            # the same combination of the filled rho, phi, psi
            F = F + m * self._grad(self._fill(C))
        F = F * self.fluid
        with np.errstate(invalid="ignore", divide="ignore"):
            u = np.where(self.fluid, (j + 0.5 * F) / np.where(self.fluid, rho, 1.0), 0.0)
        mur, mup, muq = 0.5 * (mu[0] + mu[1]), 0.5 * (mu[0] - mu[1]), mu[2] - 0.5 * (mu[0] + mu[1])
        return rho, phi, psi, j, mur, mup, muq, F, u

    def _step(self):
        rho, phi, psi, j, mur, mup, muq, F, u = self._moments3()
        cu = self.c @ u
        cF = self.c @ F
        uF = (u * F).sum(0)
        S = (1 - 0.5 / self.tf) * self.w[:, None] * (3 * (cF - uF) + 9 * cu * cF)
        fs = self.f - (self.f - self._feq(rho, u)) / self.tf + S
        gs = self.g - (self.g - self._geq(phi, mup, u)) / self.tg
        hs = self.h - (self.h - self._heq(psi, muq, u)) / self.th
        fn, gn, hn = np.zeros_like(self.f), np.zeros_like(self.g), np.zeros_like(self.h)
        F_idx = np.nonzero(self.fluid)[0]
        for i in range(self.q):
            io = self.opp[i]
            src = self.nb[io, F_idx]
            fl = self.fluid[src]
            fn[i, F_idx[fl]] = fs[i, src[fl]]
            gn[i, F_idx[fl]] = gs[i, src[fl]]
            hn[i, F_idx[fl]] = hs[i, src[fl]]
            for x, s in zip(F_idx[~fl], src[~fl]):
                cw = self.c[io] @ self._body_u(x, s, io)
                fn[i, x] = fs[io, x] - 6 * self.w[io] * rho[x] * cw
                gn[i, x] = gs[io, x] - 6 * self.w[io] * phi[x] * cw
                hn[i, x] = hs[io, x] - 6 * self.w[io] * psi[x] * cw
        self.f, self.g, self.h = fn, gn, hn
        self.t += 1

    def observe(self):
        rho, phi, psi, j, mur, mup, muq, F, u = self._moments3()
        return {"rho": self._user(rho), "phi": self._user(phi), "psi": self._user(psi),
                "ux": self._user(u[0]), "uy": self._user(u[1]), "uz": self._user(u[2]),
                "mu_rho": self._user(mur), "mu_phi": self._user(mup), "mu_psi": self._user(muq)}

    def populations(self):
        f, g = super().populations()
        return f, g, np.stack([self._user(self.h[i]) for i in range(self.q)])

"""Exact Riemann solver for the 1D Euler equations of an ideal gas.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Textbook construction: the
star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the
shock (Rankine-Hugoniot) branch for p > p_K and the isentropic rarefaction
branch otherwise; gamma = 1 uses the isothermal limits of both branches.

The paper uses this solution as the reference for its shock-tube runs
(Sec. 4, the Rankine-Hugoniot relations for u_shock and u_post, and Table
tableRankine for p_post/p_pre against p_L/p_R at equal temperatures).  For the
thermal D1Q5 model the heat-capacity ratio is gamma = (d + 2)/d = 3 in 1D.
"""
import math
from dataclasses import dataclass


@dataclass
class StarState:
    p: float
    u: float
    rho_l: float
    rho_r: float
    left_shock: bool
    right_shock: bool


def _branch(p, rho_k, p_k, gamma):
    """(f_K(p), f_K'(p)) for one side."""
    if p > p_k:  # shock
        if gamma == 1.0:
            s = math.sqrt(rho_k * p)
            f = (p - p_k) / s
            df = 1.0 / s - 0.5 * (p - p_k) / (s * p)
            return f, df
        a = 2.0 / ((gamma + 1.0) * rho_k)
        b = (gamma - 1.0) / (gamma + 1.0) * p_k
        q = math.sqrt(a / (p + b))
        return (p - p_k) * q, q * (1.0 - 0.5 * (p - p_k) / (p + b))
    c = math.sqrt(gamma * p_k / rho_k)
    if gamma == 1.0:
        return c * math.log(p / p_k), c / p
    e = (gamma - 1.0) / (2.0 * gamma)
    return (2.0 * c / (gamma - 1.0)) * ((p / p_k) ** e - 1.0), \
        (1.0 / (rho_k * c)) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))


def star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma, tol=1e-15):
    """Newton iteration for p*, then u* and the two star densities."""
    p = 0.5 * (p_l + p_r)
    for _ in range(200):
        fl, dl = _branch(p, rho_l, p_l, gamma)
        fr, dr = _branch(p, rho_r, p_r, gamma)
        g = fl + fr + (u_r - u_l)
        step = g / (dl + dr)
        p_new = max(p - step, 1e-14 * p)
        if abs(p_new - p) <= tol * p:
            p = p_new
            break
        p = p_new
    fl, _ = _branch(p, rho_l, p_l, gamma)
    fr, _ = _branch(p, rho_r, p_r, gamma)
    u = 0.5 * (u_l + u_r) + 0.5 * (fr - fl)
    return StarState(p, u, _star_rho(p, rho_l, p_l, gamma),
                     _star_rho(p, rho_r, p_r, gamma), p > p_l, p > p_r)


def _star_rho(p, rho_k, p_k, gamma):
    if gamma == 1.0:
        return rho_k * p / p_k
    if p > p_k:
        g = (gamma - 1.0) / (gamma + 1.0)
        return rho_k * (p / p_k + g) / (g * p / p_k + 1.0)
    return rho_k * (p / p_k) ** (1.0 / gamma)


def wave_speeds(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    """Left rarefaction head/tail and right shock speed for the standard
    configuration (high pressure on the left)."""
    s = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    c_l = math.sqrt(gamma * p_l / rho_l)
    c_r = math.sqrt(gamma * p_r / rho_r)
    if gamma == 1.0:
        tail = s.u - c_l
    else:
        tail = s.u - c_l * (s.p / p_l) ** ((gamma - 1.0) / (2.0 * gamma))
    shock = u_r + c_r * math.sqrt((gamma + 1.0) / (2.0 * gamma) * s.p / p_r
                                  + (gamma - 1.0) / (2.0 * gamma))
    return {"head": u_l - c_l, "tail": tail, "shock": shock, "star": s}


def pressure_ratio_table(p_ratio, gamma):
    """p_post/p_pre of the shock for a tube with p_L/p_R = p_ratio at equal
    temperatures and zero velocity (the quantity of Table tableRankine)."""
    s = star_state(p_ratio, 0.0, p_ratio, 1.0, 0.0, 1.0, gamma)
    return s.p / 1.0


def sample(x_over_t, rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    """(rho, u, p) of the self-similar solution at x/t, for a left
    rarefaction and a right shock (high pressure on the left)."""
    w = wave_speeds(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    s = w["star"]
    c_l = math.sqrt(gamma * p_l / rho_l)
    if x_over_t <= w["head"]:
        return rho_l, u_l, p_l
    if x_over_t < w["tail"]:
        if gamma == 1.0:
            u = x_over_t + c_l
            rho = rho_l * math.exp(-(u - u_l) / c_l)
            return rho, u, rho * p_l / rho_l
        g1 = gamma - 1.0
        u = 2.0 / (gamma + 1.0) * (c_l + 0.5 * g1 * u_l + x_over_t)
        c = 2.0 / (gamma + 1.0) * (c_l + 0.5 * g1 * (u_l - x_over_t))
        rho = rho_l * (c / c_l) ** (2.0 / g1)
        return rho, u, p_l * (c / c_l) ** (2.0 * gamma / g1)
    if x_over_t < s.u:
        return s.rho_l, s.u, s.p
    if x_over_t < w["shock"]:
        return s.rho_r, s.u, s.p
    return rho_r, u_r, p_r

"""Multigrid cost model (oracle; test infrastructure only).

Sec. 4.4, eq. cost:total and eq. cost:equivalent: the work of n_i cycles in
units of n_L p_L, and its normalisation v by one standard V-cycle (WAS,
n_s1 = n_s2 = 1).  c_s = c_a for WAS and 2 c_a for SCG; c_k = c_a for CS-CG
and 0 otherwise; a = q for h-MG and q/2 for p-MG with q = 1/8 (global
refinement).  Reading: the symbol a of eq. cost:equivalent is r_a of
eq. cost:total.
"""


def total_work(c_s, c_k, n_s, n_sc, n_i, a, L, c_a=1.0):
    return n_i * (n_s * c_s + c_a) * (1.0 - a ** L) / (1.0 - a) + (n_i - 1) * (n_sc - n_s) * c_s + n_i * c_k


def equivalent_vcycles(smoother, krylov_top, ns1, ns2, nsc, n_i, a, L):
    c_a = 1.0
    c_s = 2.0 * c_a if smoother == 'SCG' else c_a
    c_k = c_a if krylov_top else 0.0
    return (total_work(c_s, c_k, ns1 + ns2, nsc, n_i, a, L, c_a)
            / total_work(c_a, 0.0, 2, 2, 1, a, L, c_a))


def levels_p_mg(p):
    """p-MG with p_l = 2^(l-1) up to p_L = p."""
    L, q = 1, 1
    while q < p:
        q *= 2
        L += 1
    return L

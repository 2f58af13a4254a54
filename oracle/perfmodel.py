"""The paper's memory and bandwidth overhead model (arXiv 1703.08015, Sec. 2.2-3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function is the
closed form of the equation it names, written out in the paper's symbols:
q PDFs per node, s_d bytes per PDF, a nodes per tile edge, d dimensions,
phi geometry porosity (Eq. 11), phi_t tile porosity (Eq. 17), alpha_M the
ghost-buffer allocation ratio (Sec. 3.1.1.2), s_t node-type bytes, s_ti tile
index bytes, s_gbi ghost-buffer index bytes, s_b burst size.
"""

LATTICE = {
    # q, q_s, q_d, q_t (Sec. 3.1.1.2)
    "D2Q9": (9, 4, 4, 0),
    "D3Q19": (19, 6, 12, 0),
    "D3Q27": (27, 6, 12, 8),
}


def m_node(q, s_d):
    """Eq. (9): minimum bytes stored per node."""
    return q * s_d


def b_node(q, s_d):
    """Eq. (10): minimum bytes transferred per node per step."""
    return 2 * q * s_d


def cm_memory(q, s_d, s_idx=4):
    """Eq. (13): connectivity-matrix memory overhead."""
    return (q - 1) * s_idx / m_node(q, s_d) + 1


def cm_bandwidth(q, s_d, s_idx=4):
    """Eq. (14): connectivity-matrix bandwidth overhead."""
    return (q - 1) * s_idx / b_node(q, s_d)


def fia_memory(q, s_d, phi, s_idx=4):
    """Eq. (15): fluid-index-array memory overhead."""
    return s_idx / (phi * m_node(q, s_d)) + 1


def fia_bandwidth(q, s_d, phi, s_idx=4):
    """Eq. (16): fluid-index-array bandwidth overhead."""
    return s_idx / (phi * b_node(q, s_d)) + 1


def n_tn(a, d):
    """Nodes per tile (Sec. 3)."""
    return a ** d


def t2c_memory(q, s_d, a, d, phi_t, tiles_ratio, s_t=2, s_ti=4):
    """Eq. (24): memory overhead of tiles with two copies."""
    return (2 - phi_t + (s_t + tiles_ratio * s_ti / n_tn(a, d)) / m_node(q, s_d)) / phi_t


def c_gb(lattice):
    """Sec. 3.1.1.2: C_gb = (q_s + 2 q_d + 3 q_t) / q."""
    q, qs, qd, qt = LATTICE[lattice]
    return (qs + 2 * qd + 3 * qt) / q


def c_gbi(lattice):
    """Eq. (29): C_gbi = 2 q_s + 5 q_d + 10 q_t ghost-buffer indices per tile."""
    q, qs, qd, qt = LATTICE[lattice]
    return 2 * qs + 5 * qd + 10 * qt


def tgb_memory(lattice, s_d, a, d, phi_t, alpha_m, s_t=2, s_gbi=4):
    """Eq. (30): memory overhead of tiles with ghost buffers."""
    q = LATTICE[lattice][0]
    return (1 - phi_t + (s_t + c_gbi(lattice) * s_gbi / n_tn(a, d)) / m_node(q, s_d)
            + 2 * alpha_m * c_gb(lattice) / a) / phi_t


def b_tile(q, s_d, a, d, phi_t):
    """Eq. (19): minimum transfer per tile."""
    return n_tn(a, d) * phi_t * b_node(q, s_d)


def t2c_bandwidth(q, s_d, a, d, phi_t, s_t=2, s_ti=4):
    """Eq. (35): bandwidth overhead of tiles with two copies."""
    return ((a + 2) ** d * s_t + (q - 1) * s_ti) / b_tile(q, s_d, a, d, phi_t)


def tgb_bandwidth(lattice, s_d, a, d, phi_t, s_t=2, s_gbi=4):
    """Eq. (37): bandwidth overhead of tiles with ghost buffers."""
    q = LATTICE[lattice][0]
    return ((a + 2) ** d * s_t + c_gbi(lattice) * s_gbi) / b_tile(q, s_d, a, d, phi_t)


def full_tile_bandwidth(phi_t):
    """Eq. (38): overhead of transferring whole tiles."""
    return 1.0 / phi_t - 1.0


def t2c_bandwidth_burst(q, s_d, a, d, phi_t, s_t=2, s_ti=4):
    """Eq. (41): two-copy bandwidth overhead including whole-tile transfers."""
    return t2c_bandwidth(q, s_d, a, d, phi_t, s_t, s_ti) + full_tile_bandwidth(phi_t)


def bandwidth_utilisation(mlups, q, s_d, peak_bytes_per_s):
    """Eq. (43): BU = P[MLUPS] * B_node / B_GPU over non-solid nodes."""
    return mlups * 1e6 * b_node(q, s_d) / peak_bytes_per_s

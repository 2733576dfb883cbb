"""Mg crystallography for the oracle (test infrastructure only).

Sec. 2.1: Mg is hexagonal close packed with c/a = 1.633; the tension twins
are the six {10-12}<-1011> variants; Q_alpha is the orientation matrix of
twin variant alpha. Sec. 1: the tension twin carries a shear strain 0.129 on
the twin plane along the twin direction and rotates the lattice by about 86
degrees. Table 2: elastic constants of the Mg single crystal.

Readings (the paper is silent on these):
* Cartesian crystal frame: x || [10-10], y || [-12-10], z || [0001].
* Q_alpha = 2 m m^T - I, the 180 degree rotation about the twin-plane
  normal m. For a transversely isotropic stiffness it yields the same
  twin stiffness as the ~86.6 degree rotation about the variant's <11-20>
  axis that the paper names.
* Twin eigenstrain eps0 = gamma_tw * sym(s (x) m) (the twin term of the
  plastic velocity gradient, eq. (6), integrated over a full twin).
* Rotations R map crystal-frame vectors to sample-frame vectors.
"""

import numpy as np

# Tensor-Voigt component order (tensor shear, not engineering shear).
VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))

# The six {10-12}<-1011> tension-twin variants as (plane (hkil), direction
# [uvtw]); every pair has the direction's c-component and the plane normal's
# c-component of the same sign (tension twin).
TWIN_VARIANTS_MB = (
    ((1, 0, -1, 2), (-1, 0, 1, 1)),
    ((-1, 0, 1, 2), (1, 0, -1, 1)),
    ((0, 1, -1, 2), (0, -1, 1, 1)),
    ((0, -1, 1, 2), (0, 1, -1, 1)),
    ((1, -1, 0, 2), (-1, 1, 0, 1)),
    ((-1, 1, 0, 2), (1, -1, 0, 1)),
)

C_OVER_A = 1.633        # Sec. 2.1
GAMMA_TW = 0.129        # Sec. 1 and eq. (6)
# Table 2, in Pa: C11, C12, C13, C33, C44.
MG_HEX_PA = (59.4e9, 25.6e9, 21.4e9, 61.6e9, 16.4e9)


def hcp_basis(c_over_a, a=1.0):
    """Hexagonal basis a1, a2, a3, c in the Cartesian crystal frame."""
    a1 = a * np.array([np.sqrt(3.0) / 2.0, -0.5, 0.0])
    a2 = a * np.array([0.0, 1.0, 0.0])
    a3 = -(a1 + a2)
    c = np.array([0.0, 0.0, c_over_a * a])
    return a1, a2, a3, c


def mb_direction(uvtw, c_over_a=C_OVER_A):
    """Unit vector of the Miller-Bravais direction [uvtw]."""
    u, v, t, w = uvtw
    if u + v + t != 0:
        raise ValueError("Miller-Bravais direction needs u + v + t = 0")
    a1, a2, a3, c = hcp_basis(c_over_a)
    d = u * a1 + v * a2 + t * a3 + w * c
    return d / np.linalg.norm(d)


def mb_plane_normal(hkil, c_over_a=C_OVER_A):
    """Unit normal of the Miller-Bravais plane (hkil) from the reciprocal basis."""
    h, k, i, l = hkil
    if h + k + i != 0:
        raise ValueError("Miller-Bravais plane needs h + k + i = 0")
    a1, a2, _, c = hcp_basis(c_over_a)
    vol = a1 @ np.cross(a2, c)
    b1 = np.cross(a2, c) / vol
    b2 = np.cross(c, a1) / vol
    b3 = np.cross(a1, a2) / vol
    n = h * b1 + k * b2 + l * b3
    return n / np.linalg.norm(n)


def twin_systems(c_over_a=C_OVER_A):
    """(m, s) unit vectors of the six tension-twin variants, crystal frame."""
    return [(mb_plane_normal(p, c_over_a), mb_direction(d, c_over_a))
            for p, d in TWIN_VARIANTS_MB]


def hex_stiffness_voigt(C11, C12, C13, C33, C44):
    """6x6 Voigt stiffness (engineering-shear convention) of a hexagonal
    crystal with the c axis along z; C66 = (C11 - C12) / 2."""
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = C11
    C[2, 2] = C33
    C[0, 1] = C[1, 0] = C12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = C13
    C[3, 3] = C[4, 4] = C44
    C[5, 5] = 0.5 * (C11 - C12)
    return C


def voigt_to_tensor4(Cv):
    """C_ijkl = Cv[I(ij), J(kl)] (standard Voigt map)."""
    idx = np.zeros((3, 3), dtype=int)
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        idx[i, j] = idx[j, i] = I
    C = np.empty((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    C[i, j, k, l] = Cv[idx[i, j], idx[k, l]]
    return C


def tensor4_to_voigt(C):
    Cv = np.empty((6, 6))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            Cv[I, J] = C[i, j, k, l]
    return Cv


def rotate2(T, R):
    """T'_ij = R_ia R_jb T_ab."""
    return np.einsum("ia,jb,ab->ij", R, R, T)


def rotate4(C, R):
    """C'_ijkl = R_ia R_jb R_kc R_ld C_abcd (the twin-stiffness formula of
    Sec. 2.1.2 with Q in place of R)."""
    return np.einsum("ia,jb,kc,ld,abcd->ijkl", R, R, R, R, C)


def twin_rotation(m):
    """Q = 2 m m^T - I: 180 degree rotation about the twin-plane normal."""
    return 2.0 * np.outer(m, m) - np.eye(3)


def twin_eigenstrain(m, s, gamma=GAMMA_TW):
    """eps0 = gamma * sym(s (x) m)."""
    return 0.5 * gamma * (np.outer(s, m) + np.outer(m, s))


def schmid_factor_compression(d, m, s):
    """Schmid factor of a twin system for compression along unit d: the twin
    shears in its positive sense when -(d.s)(d.m) > 0."""
    d = np.asarray(d, float) / np.linalg.norm(d)
    return -(d @ s) * (d @ m)


def mg_tables(rotations, variant_ids, C_hex=MG_HEX_PA, gamma=GAMMA_TW,
              c_over_a=C_OVER_A):
    """Per-grain sample-frame tables.

    rotations: (G, 3, 3) crystal->sample rotations.
    variant_ids: indices (0-based) into the six variants, in order.
    Returns C_grain (G,3,3,3,3), C_var (G,V,3,3,3,3) twin stiffness
    (eq. (5)'s C_twin^alpha, sample frame) and eps0 (G,V,3,3).
    """
    rotations = np.asarray(rotations, float).reshape(-1, 3, 3)
    C_crys = voigt_to_tensor4(hex_stiffness_voigt(*C_hex))
    systems = twin_systems(c_over_a)
    G, V = rotations.shape[0], len(variant_ids)
    C_grain = np.empty((G, 3, 3, 3, 3))
    C_var = np.empty((G, V, 3, 3, 3, 3))
    eps0 = np.empty((G, V, 3, 3))
    for g in range(G):
        R = rotations[g]
        C_grain[g] = rotate4(C_crys, R)
        for a, vid in enumerate(variant_ids):
            m, s = systems[vid]
            C_tw = rotate4(C_crys, twin_rotation(m))
            C_var[g, a] = rotate4(C_tw, R)
            eps0[g, a] = rotate2(twin_eigenstrain(m, s, gamma), R)
    return C_grain, C_var, eps0


# Table 5: gradient coefficient c2 along the twin-plane normal and along the
# shear direction (N = J/m).
C2_NORMAL = 2.81e-7
C2_SHEAR = 2.81e-6


def twin_gradient_tensors(rotations, variant_ids, c2n=C2_NORMAL, c2s=C2_SHEAR, c2t=None,
                          c_over_a=C_OVER_A):
    """Anisotropic gradient tensors K_a = c2n m m + c2s s s + c2t t t of the
    given variants (t = m x s; the paper gives no value along t, read as
    c2n), turned to the sample frame: (G, V, 3, 3)."""
    c2t = c2n if c2t is None else c2t
    rotations = np.asarray(rotations, float).reshape(-1, 3, 3)
    systems = twin_systems(c_over_a)
    out = np.empty((rotations.shape[0], len(variant_ids), 3, 3))
    for g in range(rotations.shape[0]):
        for a, vid in enumerate(variant_ids):
            m, s = systems[vid]
            t = np.cross(m, s)
            K = c2n * np.outer(m, m) + c2s * np.outer(s, s) + c2t * np.outer(t, t)
            out[g, a] = rotate2(K, rotations[g])
    return out

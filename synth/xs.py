"""XS atom-type labels used as input codes.

The integer codes are part of the library interface (``dsdp_atom.xs_type``).  They
follow the X-Score typing used by the AutoDock Vina scoring function (ref. [6] of
the paper, which the paper keeps unchanged in Section 2, "Binding pose search").
Only the labels live here; radii and donor/acceptor/hydrophobic properties belong
to the scoring function and are defined separately by each implementation.
"""
XS_NAMES = [
    "C_H", "C_P", "N_P", "N_D", "N_A", "N_DA", "O_P", "O_D", "O_A", "O_DA",
    "S_P", "P_P", "F_H", "Cl_H", "Br_H", "I_H", "Met_D",
]
XS_INDEX = {n: i for i, n in enumerate(XS_NAMES)}

PALETTE_T4 = tuple(XS_INDEX[n] for n in ("C_H", "C_P", "N_A", "O_A"))
PALETTE_T8 = tuple(XS_INDEX[n] for n in ("C_H", "C_P", "N_P", "N_D", "N_A", "O_A", "O_DA", "S_P"))
PALETTE_T9 = PALETTE_T8 + (XS_INDEX["N_DA"],)
PALETTE_FULL = tuple(range(len(XS_NAMES)))

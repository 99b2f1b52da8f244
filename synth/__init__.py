"""Seeded synthetic inputs for the docking path (receptors, boxes, ligand torsion trees).

This module only draws inputs: atom positions, element and XS-type labels, ligand
trees and the five workload descriptions.  It holds none of the docking method's
arithmetic (no scoring terms, no grids, no kinematics, no search), so that the
FP64 oracle and the GPU path can both consume it without sharing any compute.

The paper's own inputs (the 995-complex scPDB-derived set, the time-split PDBBind
set and DUD-E, Section 2 "Data Set preparation") are not available; these
generators stand in for them with the shapes the paper implies: a 30 A search
cube (Section 2, "Binding pose search", third modification), drug-like ligands
of 10-60 heavy atoms with 0-15 rotatable bonds, and receptors of a few thousand
heavy atoms.
"""
from .xs import (XS_NAMES, XS_INDEX, PALETTE_T4, PALETTE_T8, PALETTE_T9,
                 PALETTE_FULL)
from .receptor import make_receptor, Receptor, make_site_points, make_score_volume
from .ligand import make_ligand, Ligand
from .configs import make_config, CONFIG_NAMES, make_box, request_ligand, request_ligand_job

__all__ = [
    "XS_NAMES", "XS_INDEX", "PALETTE_T4", "PALETTE_T8", "PALETTE_T9", "PALETTE_FULL",
    "make_receptor", "Receptor", "make_site_points", "make_score_volume", "make_ligand", "Ligand", "make_config",
    "CONFIG_NAMES", "make_box", "request_ligand", "request_ligand_job",
]

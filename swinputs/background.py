"""Background amino-acid frequencies used to draw synthetic residues.

Robinson & Robinson, PNAS 88:8880 (1991), the composition NCBI BLAST uses as
its standard background, for the 20 standard residues in alphabet order
A R N D C Q E G H I L K M F P S T W Y V.  They shape the score distribution
of the synthetic workloads; no result depends on their exact values.
"""
import numpy as np

BACKGROUND_FREQS = np.array([
    0.07805, 0.05129, 0.04487, 0.05364, 0.01925, 0.04264, 0.06295, 0.07377,
    0.02199, 0.05142, 0.09019, 0.05744, 0.02243, 0.03856, 0.05203, 0.07120,
    0.05841, 0.01330, 0.03216, 0.06441,
], dtype=np.float64)
BACKGROUND_FREQS = BACKGROUND_FREQS / BACKGROUND_FREQS.sum()

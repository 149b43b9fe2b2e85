"""FP64 CPU oracle of the Plenoxels hot path (test infrastructure only)."""

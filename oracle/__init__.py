"""CPU oracle of the rod step and of the learned coarse step (test infrastructure only)."""

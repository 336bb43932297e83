"""CPU oracle of the Hough trigger path (test infrastructure only)."""

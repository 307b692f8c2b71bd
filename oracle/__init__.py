"""CPU oracle of the shadow-map shading path (test infrastructure only)."""

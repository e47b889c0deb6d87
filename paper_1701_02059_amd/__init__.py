"""MI355X-native short-range force and time-step engine for the two-component
CGMD red-cell membrane model over an adaptive Voronoi cell list (OpenRBC,
Tang et al.)."""

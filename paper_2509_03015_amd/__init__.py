"""MI355X-native solver for SPD block-tridiagonal systems by recursive Schur-complement reduction."""

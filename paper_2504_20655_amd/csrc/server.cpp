// Continuous-batching server (filled in by the serving work).

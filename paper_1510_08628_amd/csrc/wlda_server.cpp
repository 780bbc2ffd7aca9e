// placeholder: continuous-batching fold-in server (filled in next)
